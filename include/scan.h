/*
 * scan.h -- C ABI of the fused columnar scan for AMD Instinct MI355X (gfx950).
 *
 * The operation (the paper, "Problem and Model" and "Method"): read a
 * bit-packed integer column, decode every value, test a range predicate and
 * aggregate COUNT and SUM in one pass, optionally skipping 1024-value blocks
 * whose min/max zone map misses the predicate.  Results are exact integers:
 *     count = #{ i < n : lo <= v_i < hi }
 *     sum   = (sum of those v_i) mod 2^64, as two's-complement int64
 *     blocks_read = blocks whose payload the scan had to decode: all blocks
 *                   with zone maps off, #{k : not(max_k < lo or min_k >= hi)}
 *                   with zone maps on; 0 when lo >= hi.
 * Every strategy (decoder layout, branch-free or compacting predicate, zone
 * maps on or off, batched or single) gives bit-identical count and sum.
 *
 * Conventions.
 *  - No C++ types, no exceptions cross this boundary.  Every call returns a
 *    scan_status; the message of the last failure on a context is kept for
 *    scan_last_error().
 *  - "device" pointers are HIP device allocations (e.g. a torch CUDA tensor's
 *    data_ptr()); the caller owns them and keeps them alive until the call (or,
 *    for *_async and replayed batches, the stream) is done.  "host" pointers
 *    are ordinary CPU memory.
 *  - A context is bound to one device and one HIP stream and is NOT thread
 *    safe: use one context per host thread.  All GPU work of a context is
 *    enqueued on its stream.
 *
 * Column format (the paper fixes 1024-value blocks, a row-major and a
 * lane-transposed packing, byte-aligned widths that coincide with plain
 * arrays, frame-of-reference bit-unpacking and per-block zone maps; the bit
 * order and the delta/dictionary variants are this library's reading):
 *  - L = 1024 values per block, nb = ceil(n / L) blocks; block k holds
 *    32*b u32 words (b*128 bytes) starting at word 32*b*k of the payload.
 *  - SCAN_LAYOUT_RM: value j of a block occupies block bits [j*b, j*b + b);
 *    block bit t is bit (t mod 32) of block word (t div 32) (LSB first).
 *  - SCAN_LAYOUT_LI: value j goes to lane j mod 32, slot j div 32; lane bit t
 *    is bit (t mod 32) of block word 32*(t div 32) + lane, so slot s of every
 *    lane shares one word index and shift.
 *  - Tail slots (j >= n - k*L in the last block) are zero and never counted.
 *  - SCAN_ENC_FOR: v = block_ref[k] + code as u32 (block_ref NULL: all 0).
 *  - SCAN_ENC_DELTA_FOR: v = block_base[k] + d_0 + ... + d_j (int64), d_0 = 0.
 *  - SCAN_ENC_DICT: v = dict[code], dict strictly increasing int64,
 *    dict_len <= min(2^b, 4096).
 *  - Zone maps: per block, min and max over the block's valid slots of the
 *    decoded values (u32 for FOR, int64 for DELTA_FOR) or of the codes (u32,
 *    DICT).
 */
#ifndef SCAN_H
#define SCAN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SCAN_BLOCK_VALUES 1024u
#define SCAN_MAX_DICT 4096u

typedef struct scan_ctx scan_ctx;

typedef enum {
  SCAN_OK = 0,
  SCAN_EINVAL = -1,       /* bad argument; nothing was enqueued */
  SCAN_ENOMEM = -2,       /* a device or host allocation failed */
  SCAN_EDEVICE = -3,      /* a HIP call failed; the context may be unusable */
  SCAN_EUNSUPPORTED = -4, /* strategy not valid for this column (layout, width, missing zone maps) */
  SCAN_EBUSY = -5         /* resource temporarily exhausted (serving admission) */
} scan_status;

typedef enum { SCAN_ENC_FOR = 0, SCAN_ENC_DELTA_FOR = 1, SCAN_ENC_DICT = 2 } scan_encoding;
typedef enum { SCAN_LAYOUT_RM = 0, SCAN_LAYOUT_LI = 1 } scan_layout;

/* Half-open predicate [lo, hi) on decoded values; lo >= hi selects nothing.
 * Equality v == x is [x, x+1); v < c on unsigned data is [0, c). */
typedef struct {
  int64_t lo, hi;
} scan_predicate;

enum { SCAN_AGG_COUNT = 1u, SCAN_AGG_SUM = 2u };

/* Strategy = decoder | (predicate mode << 2) | (zone maps << 3) | (all-match << 4).
 *  decoder SCAN_DEC_RM_LDS:    row-major; a wavefront stages each block in LDS
 *                              and extracts values with funnel shifts;
 *  decoder SCAN_DEC_RM_DIRECT: row-major; each lane loads its own 32-value slice
 *                              (b words) into registers, constant shifts;
 *  decoder SCAN_DEC_LI:        lane-interleaved layout, register decode;
 *  decoder SCAN_DEC_BYTES:     b in {8,16,32}, FOR, row-major read as a plain array.
 *  mode SCAN_PRED_BF:  branch-free: every value is tested and added under a mask;
 *  mode SCAN_PRED_SV:  wavefront selection-vector compaction (ballot + mbcnt)
 *                      into LDS, aggregated over the compacted list.
 *  SCAN_ALL_MATCH (with zone maps and block_sum): a block whose [min, max] lies
 *                      inside [lo, hi) is not decoded; it adds its valid-value
 *                      count to COUNT and block_sum[k] to SUM, and does not count
 *                      in blocks_read (which then counts decoded blocks only).
 * SCAN_STRAT_AUTO lets the library choose (learned selector if loaded, else a
 * fixed heuristic). */
enum {
  SCAN_DEC_RM_LDS = 0,
  SCAN_DEC_RM_DIRECT = 1,
  SCAN_DEC_LI = 2,
  SCAN_DEC_BYTES = 3,
  SCAN_PRED_BF = 0,
  SCAN_PRED_SV = 1,
  SCAN_ALL_MATCH = 16,
  SCAN_STRAT_AUTO = -1
};
#define SCAN_STRATEGY(dec, sv, zm) ((int32_t)((dec) | ((sv) << 2) | ((zm) << 3)))

typedef struct {
  const uint32_t* payload;    /* device: nb*32*b words, 16-byte aligned */
  const uint32_t* block_ref;  /* device: FOR references (nb u32) or NULL for all-zero */
  const int64_t* block_base;  /* device: DELTA_FOR bases (nb int64) */
  const int64_t* dict;        /* device: DICT entries */
  uint32_t dict_len;
  uint32_t layout;            /* scan_layout */
  const void* zone_min;       /* device: nb entries (u32, or int64 for DELTA_FOR); NULL = none */
  const void* zone_max;
  uint64_t n;                 /* values in the column */
  const uint64_t* block_sum;  /* device: nb sums of each block's decoded values mod 2^64, or NULL */
} scan_column;

typedef struct {
  uint64_t count;
  int64_t sum;
  uint64_t blocks_read;
  uint64_t blocks_total;
  int32_t strategy_used;
  int32_t status;             /* scan_status of this item (batch and serving results) */
} scan_result;

typedef struct {
  scan_column col;
  int32_t enc;                /* scan_encoding */
  uint32_t b;                 /* bits per code, 1..32 */
  scan_predicate pred;
  uint32_t agg;               /* SCAN_AGG_* bits; COUNT is always produced */
  int32_t strategy;           /* SCAN_STRATEGY(...) or SCAN_STRAT_AUTO */
} scan_item;

/* Launch tuning of one (encoding, width, strategy): work-group size (64, 128,
 * 192 or 256), work-groups per compute unit (0 = as many as fit), the
 * window: wavefronts take grid-strided windows of this many consecutive
 * blocks (1..64; 0 = one pipelined decode step), and the step depth (values
 * each wavefront has in flight per pipelined step): 0 the kernel's default,
 * 1 its alternative.  The alternative exists for the branch-free
 * frame-of-reference kernels of the register decoders (SCAN_DEC_RM_DIRECT,
 * SCAN_DEC_LI) without block references (half as many block pairs per step
 * below b = 16, one pair more at b = 16-23, one pair instead of two from
 * b = 24 on) and for the branch-free dictionary kernels of SCAN_DEC_RM_DIRECT
 * (below b = 16 their default is the shallower step and the alternative
 * twice as deep; above, as for frame of reference); other kernels ignore it.  Zero fields mean "library
 * default". */
typedef struct {
  int32_t wg_size;
  int32_t wgs_per_cu;
  int32_t window_blocks;
  int32_t depth;
} scan_tune;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device` enqueuing on `hip_stream`
 * (a hipStream_t, or NULL for the null stream).  Allocates the context's
 * device scratch (partials, counters, result slots). */
scan_status scan_create(scan_ctx** out, int device, void* hip_stream);
/* Change the stream later calls enqueue on.  The new stream is first made to
 * wait (an event, no host wait) for the work already enqueued on the old one,
 * since every scan of a context writes the same device partials and result
 * slot.  HIP failure -> SCAN_EDEVICE (the stream is then unchanged). */
scan_status scan_set_stream(scan_ctx* ctx, void* hip_stream);
/* Waits for the context's stream, then frees everything the context owns. */
void scan_destroy(scan_ctx* ctx);
/* Message of the last failed call on ctx ("" if none).  Valid until the next call. */
const char* scan_last_error(const scan_ctx* ctx);
/* Number of compute units of the context's device. */
int scan_device_cus(const scan_ctx* ctx);

/* ------------------------------------------------------------------ scans */

/* Scan one column and wait for the result (written to *out, host memory).
 * Errors: b outside 1..32, NULL payload, misaligned payload, missing
 * references/bases/dictionary for the encoding, dict_len > min(2^b, 4096)
 * -> SCAN_EINVAL; strategy not valid for the column -> SCAN_EUNSUPPORTED.
 * n == 0 or lo >= hi -> SCAN_OK with zero count and sum. */
scan_status scan_run(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b,
                     const scan_predicate* pred, uint32_t agg, int32_t strategy, scan_result* out);

/* Enqueue one scan on the context stream; the result lands in *out_dev
 * (device memory, one scan_result) when the stream reaches it.  No host sync;
 * scan_sync() waits.  SCAN_STRAT_AUTO resolves to the heuristic here (no sync). */
scan_status scan_run_async(scan_ctx* ctx, const scan_item* item, scan_result* out_dev);
scan_status scan_sync(scan_ctx* ctx);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): scan_run_async without a
 * context and without any allocation.  The same kernels run with the library
 * default launch shapes (no per-context tuning; SCAN_STRAT_AUTO resolves to
 * the heuristic), enqueued on hip_stream (a hipStream_t, or NULL) of the
 * current HIP device; the result (one scan_result, every field, status 0)
 * lands in *out_dev (device memory) when the stream reaches it.  No host
 * sync.  The work-group partials live in a static device array of the
 * library, SCAN_STATIC_MAX_WORKGROUPS x 32 bytes per device (128 KiB, held
 * until the process ends; set up on the first call on each device); launches
 * are capped to that many work-groups, so any column length is accepted.
 * Every call on a device shares that array: calls that overlap on one device
 * (different streams, or several host threads) race and give wrong results;
 * calls in one stream's order do not.  Errors: the argument checks of
 * scan_run -> SCAN_EINVAL / SCAN_EUNSUPPORTED before anything is enqueued;
 * HIP failures -> SCAN_EDEVICE.  There is no message (no context). */
#define SCAN_STATIC_MAX_WORKGROUPS 4096u
scan_status scan_run_static(const scan_item* item, void* hip_stream, scan_result* out_dev);

/* Set / read the launch tuning used for (enc, b, strategy). */
scan_status scan_set_tune(scan_ctx* ctx, int32_t enc, uint32_t b, int32_t strategy, const scan_tune* t);
scan_status scan_get_tune(scan_ctx* ctx, int32_t enc, uint32_t b, int32_t strategy, scan_tune* t);

/* Autotuner: times every launch configuration of a small grid (work-group
 * size {64,128,256} x work-groups per CU {1,2,4,8} x window {2,4,8,16,64}
 * blocks x step depth {0, 1} where the kernel has the alternative depth) for
 * one column and strategy, median of `reps` runs each with HIP events on
 * the context stream (a 512 MiB read before each run keeps the column out of
 * the 256 MB last-level cache), and keeps the fastest with scan_set_tune.
 * *out (host, may be NULL) receives it, *ms_out (may be NULL) its time in ms.
 * The context allocates its 512 MiB eviction buffer on first use. */
scan_status scan_autotune(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b,
                          const scan_predicate* pred, int32_t strategy, int32_t reps, scan_tune* out, float* ms_out);
/* Persist / restore every tuning of the context as JSON (one entry per line).
 * scan_tune_load installs nothing and returns SCAN_EINVAL when the file cannot
 * be read, holds no entry, or has an entry line that does not parse or holds
 * an invalid tuning (the message names the line). */
scan_status scan_tune_save(scan_ctx* ctx, const char* path);
scan_status scan_tune_load(scan_ctx* ctx, const char* path);

/* ------------------------------------------------------------- run length */
/* Run-length encoding (the paper, "Method": implemented there alongside the
 * bit-packed decoders, no result reported; the format below is this
 * library's).
 * Run-length encoded u32 column: runs never cross a 1024-value block; run r
 * has value run_value[r] and length run_len[r] (1..1024); block k owns runs
 * block_run[k] .. block_run[k+1]-1.  The scan tests the predicate once per run
 * and adds the run's length to COUNT and value x length to SUM (mod 2^64). */
typedef struct {
  const uint32_t* run_value;  /* device, 16-byte aligned */
  const uint16_t* run_len;    /* device, 8-byte aligned */
  const uint64_t* block_run;  /* device: nb + 1 entries */
  const uint32_t* zone_min;   /* device: per-block min / max of the values, or NULL */
  const uint32_t* zone_max;
  uint64_t n;                 /* values (sum of the run lengths) */
} scan_rle_column;

/* Synchronous scan; flags: bit 0 zone maps, bit 1 with bit 0 the all-match
 * shortcut (a block inside the predicate is taken whole).  Same result
 * contract as scan_run; strategy_used reports the flags.  Errors: flags
 * outside 0..3, NULL or misaligned run arrays (n > 0) -> SCAN_EINVAL; zone
 * maps requested without them -> SCAN_EUNSUPPORTED. */
scan_status scan_run_rle(scan_ctx* ctx, const scan_rle_column* col, const scan_predicate* pred, uint32_t flags,
                         scan_result* out);
/* Enqueue the same scan on the context stream; the whole result (count, sum,
 * blocks_read, blocks_total, strategy_used, status 0) lands in *out_dev
 * (device memory, one scan_result) when the stream reaches it.  No host sync;
 * scan_sync() waits.  Validation errors return before anything is enqueued. */
scan_status scan_run_rle_async(scan_ctx* ctx, const scan_rle_column* col, const scan_predicate* pred,
                               uint32_t flags, scan_result* out_dev);

/* ------------------------------------------------------ materializing select */
/* The ascending positions (u32 row indices) of the rows with lo <= v < hi,
 * written to positions (device, capacity entries) -- the materializing scan
 * whose cost the paper's branch crossover concerns -- and late
 * materialization on a position list.  Frame-of-reference (with or without
 * block references) and dictionary columns, row-major, n < 2^32.
 * flags: bit 0 zone maps (skip blocks that cannot match), bit 1 with bit 0 the
 * all-match shortcut (a block inside the predicate writes its position range
 * without being read).  Synchronous.  *n_selected (host) always receives the
 * number of matches; if it exceeds capacity nothing is written and the call
 * returns SCAN_ENOMEM (call again with a larger buffer).  With capacity >= n
 * the buffer holds any outcome and the passes run back to back with one wait
 * at the end; otherwise the call waits for the count before writing.
 * Positions leave in row order (two passes: per-block counts, an exclusive
 * scan, then the writes). */
scan_status scan_select(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, const scan_predicate* pred,
                        uint32_t flags, uint32_t* positions, uint64_t capacity, uint64_t* n_selected);
/* The positions of positions_in[0..n_in) (device, any order; a position >= n
 * never passes) whose value in this column lies in [lo, hi), in input order, to positions_out (device, room
 * for n_in); *n_out (host) receives how many.  Synchronous. */
scan_status scan_refine(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, const scan_predicate* pred,
                        const uint32_t* positions_in, uint64_t n_in, uint32_t* positions_out, uint64_t* n_out);
/* Decoded values at positions[0..n) into values (device int64; 0 for a
 * position >= the column's n).  Synchronous. */
scan_status scan_gather(scan_ctx* ctx, const scan_column* col, int32_t enc, uint32_t b, const uint32_t* positions,
                        uint64_t n, int64_t* values);

/* ---------------------------------------------------------------- batches */
/* Not in the paper (the workload's mixed-column batch).
 * Many columns (mixed length, width, encoding, strategy) scanned by one fixed
 * sequence of kernels, whatever the number of columns.  Planned once:
 * per-column setup, strategy selection on the device (the loaded selector for
 * SCAN_STRAT_AUTO items: zone-map features, the network, the argmin; else the
 * heuristic), and lists of the columns' work items (four windows of blocks
 * each) per class (encoding, decoder, predicate mode), in item order.  A
 * replay: one persistent kernel per class with items, walking its list on a
 * static schedule (a work-group per item, one window per wavefront;
 * dictionary classes hold the column's dictionary in LDS).
 * Columns must be row-major;
 * explicit strategies must use the SCAN_DEC_RM_LDS or SCAN_DEC_RM_DIRECT
 * decoder.  Results equal scan_run's for every item, bit for bit.
 *
 * scan_batch_prepare validates the items, uploads their descriptors, windows
 * and zone-map segments once, and plans the batch on the device once: every
 * SCAN_STRAT_AUTO item's strategy (the selector's choice, from the columns'
 * zone maps as they are now, else the heuristic) and the per-class work
 * lists.  A selector choice that would add a class scan (decoder x mode of
 * the encoding) that no other column of the batch needs is taken back to the
 * heuristic when the network's predicted gains of all the columns it moves
 * into that class add up to less than the class-scan cost
 * (scan_batch_set_class_cost); so a batch's AUTO strategy can differ from
 * scan_run's for the same item.  It then captures the replay sequence (reset
 * of the result slots, then one persistent kernel per class with items) into
 * a HIP graph (see scan_batch_set_graph; if capture fails, replays enqueue
 * the kernels one by one: same results).  Baked in at that moment: the
 * strategies, and the tuning stored for (enc -1, b 0, strategy -1)
 * (work-groups per CU of the class kernels, default 4, at most the number
 * that fit, and the window, default and at most 64 blocks).  The columns'
 * contents and zone maps must not change while the batch lives.  An invalid
 * item does not fail the call: its result carries the error in `status`.
 * `items` (host) may be freed after the call; the columns' device buffers
 * must stay alive until the handle is released.  Synchronizes the context
 * stream.  *handle (host) receives an id.  Up to 2^24 items; more ->
 * SCAN_EINVAL. */
scan_status scan_batch_prepare(scan_ctx* ctx, const scan_item* items, size_t n_items, uint64_t* handle);
/* Enqueue the batch on the context stream (one graph launch).  With out
 * (host, n_items results) non-NULL, also copies the results back, waits and
 * fills it; with out NULL, only enqueues.  May be replayed any number of
 * times; replays on one context's stream run one after another. */
scan_status scan_batch_replay(scan_ctx* ctx, uint64_t handle, scan_result* out);
/* Wait for the stream and free the batch's buffers and graph. */
scan_status scan_batch_release(scan_ctx* ctx, uint64_t handle);
/* prepare + replay + release. */
scan_status scan_batch_run(scan_ctx* ctx, const scan_item* items, size_t n_items, scan_result* out);
/* Launch tuning of the batch class kernels (wgs_per_cu, window_blocks). */
scan_status scan_batch_set_tune(scan_ctx* ctx, const scan_tune* t);
/* Autotuner of the batch class kernels: for each of class-list order {0, 1}
 * x work-groups per CU {1, 2, 4, 8} x window {16, 32, 64} blocks, prepares
 * the batch (graph mode as set), replays it once, then times `reps` replays
 * (at most 16) with HIP events, each after the 512 MiB cache-evicting read
 * (allocated on first use, as for scan_autotune), and keeps the
 * median-fastest configuration as the batch tuning (scan_batch_set_tune)
 * and list order (scan_batch_set_order).  *out / *ms_out (host, may be
 * NULL) receive it (out->depth: the list order) and its time.  Results never depend on the tuning.  An
 * empty batch -> SCAN_EINVAL; on failure the previous tuning is restored. */
scan_status scan_batch_autotune(scan_ctx* ctx, const scan_item* items, size_t n_items, int32_t reps, scan_tune* out,
                                float* ms_out);
/* How later scan_batch_prepare calls build the replay: 0 direct launches,
 * 1 (the default) one graph with the class scans in sequence, 2 one graph
 * with the class scans forked over up to four branches (measured slower on
 * MI355X: the concurrent class scans contend).  Results are the same.
 * Other values -> SCAN_EINVAL. */
scan_status scan_batch_set_graph(scan_ctx* ctx, int32_t mode);
/* Order of the class lists of later scan_batch_prepare calls: 0 item order
 * (columns in the batch's order, each column's work items in block order),
 * 1 (the default) that order walked with a stride: list position j takes
 * item (j * (2^31 - 1)) mod L of the L items, which spreads every column's
 * items over the static schedule.  Deterministic either way; results are the
 * same, the speed differs with the mix (the batch autotuner tries both).
 * Other values -> SCAN_EINVAL. */
scan_status scan_batch_set_order(scan_ctx* ctx, int32_t order);
/* Cost in microseconds of one more class scan in a replay (its launch and
 * drain; default 10, measured on MI355X with 4096-column batches), used by
 * later scan_batch_prepare calls to take back selector choices that would
 * need a class scan of their own (see scan_batch_prepare).  0 keeps every
 * choice.  Negative or not finite -> SCAN_EINVAL. */
scan_status scan_batch_set_class_cost(scan_ctx* ctx, float us);
typedef struct {
  int32_t captured;           /* 0: direct launches; 1: one graph launch; 2: one graph, forked class scans */
  uint32_t kernels;           /* kernels in one replay (0 for an empty batch) */
  uint32_t class_mask;        /* class scans launched (bit enc*4 + decoder*2 + mode) */
  uint32_t work_items;        /* work items of the batch's columns */
  uint32_t pruned;            /* selector choices taken back to the heuristic (class-scan cost) */
  uint32_t reserved;
} scan_batch_stats;
/* Plan facts of a prepared batch into *out (host).  Unknown handle -> SCAN_EINVAL. */
scan_status scan_batch_info(scan_ctx* ctx, uint64_t handle, scan_batch_stats* out);

/* --------------------------------------------------------------- selector */
/* Not in the paper (the workload's learned strategy choice).
 * The strategy selector is a fully connected fp32 network 6 -> 64 -> 64 -> 8
 * (ReLU after both hidden layers) predicting a log-time for each of the eight
 * row-major strategies: class c = decoder (c & 1: RM_LDS or RM_DIRECT),
 * predicate mode ((c >> 1) & 1), zone maps ((c >> 2) & 1).  The library picks
 * the class of smallest prediction among those valid for the column (zone-map
 * classes need zone maps; ties to the lowest class), subject to the fallback
 * margin below.  Parameters: W1[64][6],
 * b1[64], W2[64][64], b2[64], W3[8][64], b3[8], row-major, in that order. */
int scan_mlp_param_count(void);
/* Install parameters (host, scan_mlp_param_count() finite floats). */
scan_status scan_selector_set(scan_ctx* ctx, const float* theta_host, size_t count);
/* Back to the heuristic. */
scan_status scan_selector_clear(scan_ctx* ctx);
int scan_selector_loaded(const scan_ctx* ctx);
/* Text file: "scan-mlp-v1 <count>" then the parameters, whitespace
 * separated, then optionally "margin <x>" (loading a file without it sets
 * margin 0).  Anything else -> SCAN_EINVAL. */
scan_status scan_selector_load(scan_ctx* ctx, const char* path);
scan_status scan_selector_save(scan_ctx* ctx, const char* path);
/* Fallback margin of the selector (default 0): for a column the library keeps
 * the heuristic's strategy unless the network predicts for it a log-time at
 * least `margin` above the smallest prediction among the column's valid
 * classes (then the argmin, ties to the lowest class).  Margin 0 is the plain
 * argmin.  Negative or non-finite -> SCAN_EINVAL. */
scan_status scan_selector_set_margin(scan_ctx* ctx, float margin);
/* The selector's input features of n_items columns, written to X_dev (device,
 * n_items x 6 floats, row-major), from zone maps and descriptors only:
 *   b/32, log2(n)/24, log10(max(s, 1e-6))/6 (s: selectivity estimated from the
 *   zone maps, values spread evenly over each block's [min, max]), fraction
 *   of blocks whose [min, max] meets the predicate, clustering
 *   1 - mean(max - min)/(global max - global min + 1), encoding/2.
 * Columns without zone maps get s = 1, fraction 1, clustering 0.  Synchronous. */
scan_status scan_features(scan_ctx* ctx, const scan_item* items, size_t n_items, float* X_dev);

/* Training kernels (all pointers device, fp32, enqueued on the context stream).
 * Forward: out[rows][8] = network(theta, X[rows][6]). */
scan_status scan_mlp_forward(scan_ctx* ctx, const float* theta, const float* X, uint32_t rows, float* out);
/* Masked squared error L = inv_denom * sum_{i,j} M[i][j] (out[i][j] - Y[i][j])^2
 * and its gradient w.r.t. theta (grad: param_count floats; loss: one float,
 * may be NULL).  Work space is owned by the context. */
scan_status scan_mlp_loss_grad(scan_ctx* ctx, const float* theta, const float* X, const float* Y, const float* M,
                               uint32_t rows, float inv_denom, float* grad, float* loss);
/* One Adam update (Kingma and Ba, 2015) of `count` parameters at 1-based
 * `step`, with bias correction. */
scan_status scan_adam_step(scan_ctx* ctx, float* theta, const float* grad, float* m, float* v, uint32_t count,
                           int32_t step, float lr, float beta1, float beta2, float eps);

/* ---------------------------------------------------------------- serving */
/* Not in the paper (the workload's serving loop); each query is the paper's
 * fused scan ("Method") over a conjunction of range predicates.
 * A table: columns of equal row count, each row-major frame-of-reference
 * (optional per-block references) or dictionary, any width 1..32, all with
 * zone maps.  A query: COUNT and SUM(sum_col) over the rows where every filter
 * conjunct filter_col[f] in [lo_f, hi_f) holds (1..3 conjuncts; values for FOR
 * columns, dictionary entries for dictionary columns).  Same exact-integer
 * contract as scan_run: count = #{rows passing}, sum = (sum of sum_col over
 * them) mod 2^64; blocks_read = blocks no conjunct's zone map excluded.  A
 * result never depends on the other queries of a batch. */
typedef struct {
  scan_column col;            /* device buffers, caller-owned, alive as long as the table */
  int32_t enc;                /* SCAN_ENC_FOR or SCAN_ENC_DICT */
  uint32_t b;
} scan_table_column;

typedef struct scan_table scan_table;
typedef struct scan_server scan_server;

typedef struct {
  uint32_t n_filters;         /* 1..3 */
  uint32_t filter_col[3];
  scan_predicate filter[3];
  uint32_t sum_col;
  uint32_t reserved;
} scan_query;

typedef struct {
  uint64_t ticket;            /* scan_server_submit's ticket (scan_query_run: the query's index) */
  uint64_t count;
  int64_t sum;
  uint64_t blocks_read;
  double submit_us, done_us;  /* host steady clock (scan_server_clock_us): submission, completion seen */
  int32_t status;
  int32_t reserved;
} scan_query_result;

/* Server knobs.  Admission: a submit returns SCAN_EBUSY when max_inflight
 * queries are admitted and unfinished, or when one more would take the
 * device workspace of admitted queries (a descriptor and two result slots,
 * 184 bytes each) past hbm_budget_bytes.  Batching: a free stream launches the
 * oldest pending queries (at most max_batch) when the batch is full, when the
 * oldest has waited batch_window_us, when no stream is busy, or when a stream
 * has just completed.  window_blocks (0 = 64, at most 64) and wgs_per_cu
 * (0 = as many as fit on a CU) shape the kernel launch. */
typedef struct {
  uint64_t hbm_budget_bytes;
  uint32_t max_inflight;
  uint32_t n_streams;         /* 1..16 streams of default priority */
  uint32_t max_batch;
  uint32_t batch_window_us;
  uint32_t window_blocks;
  uint32_t wgs_per_cu;
  uint32_t kernel;            /* SCAN_QUERY_PER_QUERY (0, default) or SCAN_QUERY_SHARED (1) */
  uint32_t reserved;
} scan_server_config;

/* Validate the columns and upload their descriptors.  Errors: different row
 * counts, missing zone maps, delta columns or LI layout -> SCAN_EINVAL /
 * SCAN_EUNSUPPORTED. */
scan_status scan_table_create(scan_ctx* ctx, const scan_table_column* cols, uint32_t n_cols, scan_table** out);
void scan_table_destroy(scan_table* t);
/* Run n queries as one batch on the context stream and wait; out (host) gets
 * n results.  Bad filter or sum column indices -> SCAN_EINVAL. */
scan_status scan_query_run(scan_ctx* ctx, const scan_table* t, const scan_query* queries, size_t n,
                           scan_query_result* out);
/* Launch shape of scan_query_run (0 = default: 64-block windows for the
 * per-query kernel, 8 for the shared one; as many work-groups per CU as fit). */
scan_status scan_query_set_tune(scan_ctx* ctx, int32_t wgs_per_cu, int32_t window_blocks);
/* Which query kernel scan_query_run uses (the server takes it from its config):
 *  SCAN_QUERY_PER_QUERY (default): a work item is (window, query); each query
 *    stages the blocks it needs itself, and the window-major item order lets
 *    the queries of a batch share column reads through the caches;
 *  SCAN_QUERY_SHARED: a work item is a window of blocks for every query of
 *    the batch; per block, every column block that any surviving query needs
 *    is read once into LDS and all of them are evaluated on it (tables of at
 *    most 64 columns whose blocks fit 64 KiB together; 64 queries per
 *    launch).  It reads 3.3x fewer bytes but measured slower on MI355X
 *    (10.9 against 6.0 ms for 64 queries on 16 x 2^28 rows): each wavefront
 *    runs its share of the queries one after another between two barriers.
 * Same results.  Other values -> SCAN_EINVAL.  A table the shared kernel
 * cannot hold always runs the per-query kernel. */
enum { SCAN_QUERY_PER_QUERY = 0, SCAN_QUERY_SHARED = 1 };
scan_status scan_query_set_kernel(scan_ctx* ctx, int32_t kernel);

/* Start a server on the context's device (its own host thread and streams;
 * the context itself is not used by the thread).  The table must outlive it. */
scan_status scan_server_create(scan_ctx* ctx, const scan_table* t, const scan_server_config* cfg, scan_server** out);
/* Thread-safe.  SCAN_EBUSY: not admitted (retry later); *ticket identifies it. */
scan_status scan_server_submit(scan_server* s, const scan_query* q, uint64_t* ticket);
/* Thread-safe.  Moves up to max finished results to out, waiting up to wait_us
 * for the first; *n_out receives how many. */
scan_status scan_server_poll(scan_server* s, scan_query_result* out, size_t max, size_t* n_out, uint32_t wait_us);
/* stats4: batches launched, queries launched, admitted unfinished, pending. */
scan_status scan_server_stats(scan_server* s, uint64_t* stats4);
/* The clock of submit_us / done_us, in microseconds. */
double scan_server_clock_us(void);
/* Stops the thread, waits for launched batches; pending queries are dropped. */
void scan_server_destroy(scan_server* s);

/* Host-only discrete-event run of the same admission and batching policy:
 * arrivals at arrival_us[0..n) (non-decreasing), a batch of q queries busy
 * for batch_fixed_us + q * per_query_us on its stream.  Writes per query the
 * launch and completion times and the admission status (SCAN_EBUSY: refused,
 * times -1), and the number of batches.  Needs no GPU. */
scan_status scan_serve_simulate(const scan_server_config* cfg, const double* arrival_us, size_t n,
                                double batch_fixed_us, double per_query_us, double* launch_us, double* done_us,
                                int32_t* status, uint64_t* n_batches);

/* -------------------------------------------------------------- encoders */
/* Host-side encoders (host pointers).  Payload buffers must hold
 * scan_payload_words(n, b) u32; zone-map and reference/base buffers nb entries.
 * They are written from the format text above, independently of any checker. */
uint64_t scan_payload_words(uint64_t n, uint32_t b);
/* FOR: ref_policy 0 = all references 0, 1 = per-block minimum (block_ref must
 * then be non-NULL).  Fails with SCAN_EINVAL if a value does not fit b bits
 * above its reference.  zone_min/zone_max may be NULL. */
scan_status scan_encode_for(const uint32_t* values, uint64_t n, uint32_t b, uint32_t layout,
                            int32_t ref_policy, uint32_t* payload, uint32_t* block_ref,
                            uint32_t* zone_min, uint32_t* zone_max);
/* DELTA_FOR: values non-decreasing; every difference must fit b bits. */
scan_status scan_encode_delta(const int64_t* values, uint64_t n, uint32_t b, uint32_t* payload,
                              int64_t* block_base, int64_t* zone_min, int64_t* zone_max);
/* DICT: codes (indices into a dictionary of dict_len entries) packed row-major. */
scan_status scan_encode_dict(const uint32_t* codes, uint64_t n, uint32_t b, uint32_t dict_len,
                             uint32_t* payload, uint32_t* zone_min, uint32_t* zone_max);
/* Run-length encoder (host pointers): run_value / run_len hold up to n runs,
 * block_run nb + 1 entries, zone_min / zone_max nb entries (may be NULL);
 * *n_runs receives the number of runs. */
scan_status scan_rle_encode(const uint32_t* values, uint64_t n, uint32_t* run_value, uint16_t* run_len,
                            uint64_t* block_run, uint32_t* zone_min, uint32_t* zone_max, uint64_t* n_runs);
/* Per-block sums for the all-match shortcut (an extension of the paper's
 * per-block zone maps, "Method"; not in the paper).
 * Per-block sums of decoded values mod 2^64 (host pointers; out has nb
 * entries) for scan_column.block_sum: enc SCAN_ENC_FOR takes u32 values,
 * SCAN_ENC_DELTA_FOR int64 values, SCAN_ENC_DICT u32 codes and the dictionary
 * (dict_len entries; a code >= dict_len -> SCAN_EINVAL). */
scan_status scan_block_sums(int32_t enc, const void* values, uint64_t n, const int64_t* dict, uint32_t dict_len,
                            uint64_t* out);

/* ----------------------------------------------------- bandwidth probes */
/* The paper measures beta per machine as the empirical sequential-read
 * maximum (buffers much larger than the last-level cache) and reports STREAM
 * triad beside it ("Method"); these probes measure both on the device.
 * Streaming read of `bytes` (multiple of 16) from `buf` (device) with 16-byte
 * loads; `wgs` work-groups of `wg_size` threads (0 = defaults); `unroll`
 * independent loads in flight per thread (1, 2, 4 or 8).  Writes a checksum
 * into sink[0] (device u64) so the reads cannot be elided.  Enqueue only. */
scan_status scan_beta_read(scan_ctx* ctx, const void* buf, uint64_t bytes, int32_t wgs,
                           int32_t wg_size, int32_t unroll, uint64_t* sink);
/* STREAM triad a[i] = b[i] + s*c[i] over n floats (device). Enqueue only. */
scan_status scan_beta_triad(scan_ctx* ctx, float* a, const float* b, const float* c, float s,
                            uint64_t n);
/* Read `bytes` (multiple of 16) of device scratch `buf` so that later reads
 * of other data miss the caches; the lines it leaves cached are clean, so no
 * write-back competes with the next kernel.  Use a buffer several times the
 * 256 MiB last-level cache.  The contents of `buf` are left as they were, except
 * that its first 16 bytes may be overwritten.  Enqueue only. */
scan_status scan_cache_flush(scan_ctx* ctx, void* buf, uint64_t bytes);

#ifdef __cplusplus
}
#endif
#endif /* SCAN_H */

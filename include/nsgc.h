/*
 * nsgc.h -- per-window traffic-matrix statistics on AMD Instinct MI355X (gfx950).
 *
 * The operation (arXiv 2509.03653, Section IV "Graph Analytics", Table III;
 * the reverse queries swap src and dst, Table III caption).  A window is a
 * multiset of (src, dst) packets with 32-bit anonymized addresses; its traffic
 * matrix A counts packets per pair, A(s,d) = #{packets with src s, dst d}
 * (the packets form a multigraph, Section V).  With row sums r(s), row
 * non-zero counts f(s), column sums c(d) and column non-zero counts g(d):
 *
 *   valid_packets           = sum of A                 (Table III, row 1)
 *   unique_links            = nnz(A)                   (row 2)
 *   max_link_packets        = max of A                 (row 4)
 *   unique_sources          = #{s : r(s) > 0}          (row 5)
 *   max_source_packets      = max r                    (row 7)
 *   max_source_fanout       = max f                    (row 9)
 *   unique_destinations     = #{d : c(d) > 0}          (row 5, reversed)
 *   max_destination_packets = max c                    (row 7, reversed)
 *   max_destination_fanin   = max g                    (row 9, reversed)
 *
 * A window whose valid_packets comes back with bit 63 set hit an internal
 * limit of the library (it never happens for windows below 2^32 packets
 * unless the library is broken); its statistics must not be used.
 *
 * Maxima over an empty set are 0: an empty window yields nine zeros.  Every
 * pair in a window is a valid packet (there is no validity mask at this layer).
 * All results are exact integers; they do not depend on batching, tiering,
 * tuning or the order of packets.
 *
 * Conventions for every entry point:
 *   - src, dst: DEVICE pointers to uint32 arrays, caller-owned, read-only;
 *     packet i is (src[i], dst[i]).
 *   - window_offsets: HOST pointer to num_windows+1 int64 values, caller-owned,
 *     read during the call only.  Window w is packets
 *     [window_offsets[w], window_offsets[w+1]).  Offsets must be >= 0 and
 *     non-decreasing; offsets[0] may be non-zero; empty windows are legal.
 *     A window may hold at most 2^32 - 1 packets.
 *   - out_stats: DEVICE pointer to num_windows nsgc_stats (8-byte aligned),
 *     caller-owned, fully overwritten.
 *   - stream: the HIP stream the work is enqueued on (0 = null stream).  The
 *     call returns after enqueueing; results are valid once the stream has
 *     reached that point.  Input buffers must stay alive and unmodified until
 *     then.  One exception: a batch with a window of the large-window tier
 *     (nsgc_tune.large_min_log2) waits once per such window for the stream,
 *     to read back the window's link count, so the call returns only after
 *     the work enqueued before that point has run.
 *   - Argument errors are reported synchronously with nothing enqueued and
 *     out_stats untouched.  A HIP runtime failure returns NSGC_ERR_HIP and
 *     nsgc_last_hip_error() gives the hipError_t.
 *   - The library keeps per-(device, stream) workspaces, so calls on
 *     different streams may overlap; calls on one stream run in order.  All
 *     entry points are thread-safe: host threads calling on different
 *     streams plan and enqueue concurrently (a lock per stream, per graph
 *     object and per device's fixed scratch; the shared state is only looked
 *     up under a process-wide lock), calls on one stream take turns.
 *     nsgc_graph_destroy must not overlap a launch of the same graph.
 *   - The direct forms (nsgc_window_stats, _plain, _timed) must not be
 *     called on a stream that is being captured: they return
 *     NSGC_ERR_CAPTURING with nothing enqueued.  Their plan upload reads a
 *     staging buffer that later calls overwrite, so a replay would not be
 *     the same call.  Capture-safe batching is the graph form below.
 */
#ifndef NSGC_H_
#define NSGC_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One window's statistics, 72 bytes, in Table III order (see above). */
typedef struct nsgc_stats {
  uint64_t valid_packets;
  uint64_t unique_links;
  uint64_t max_link_packets;
  uint64_t unique_sources;
  uint64_t max_source_packets;
  uint64_t max_source_fanout;
  uint64_t unique_destinations;
  uint64_t max_destination_packets;
  uint64_t max_destination_fanin;
} nsgc_stats;

typedef enum nsgc_status {
  NSGC_OK = 0,
  NSGC_ERR_INVALID_ARG = -1,  /* null pointer, negative count, misaligned out */
  NSGC_ERR_BAD_OFFSETS = -2,  /* negative/decreasing offsets, window >= 2^32 */
  NSGC_ERR_NO_MEMORY = -3,    /* workspace allocation failed or exceeds limit */
  NSGC_ERR_HIP = -4,          /* HIP runtime error, see nsgc_last_hip_error() */
  NSGC_ERR_INTERNAL = -5,
  NSGC_ERR_CAPTURING = -6,    /* called on a stream that is being captured */
  NSGC_ERR_TOO_LARGE = -7     /* batch exceeds nsgc_window_stats_noalloc's fixed scratch */
} nsgc_status;

/*
 * Batched form.  All windows of the call are planned together and processed
 * by one sequence of persistent kernel launches: tiny windows entirely in LDS,
 * the others by hash partitioning of the packets into LDS-sized link buckets,
 * link aggregation per bucket, then row and column aggregation of the
 * de-duplicated links (Table III rows 1-9 and their reverses, per window).
 */
int nsgc_window_stats(const uint32_t* src, const uint32_t* dst,
                      const int64_t* window_offsets, int64_t num_windows,
                      nsgc_stats* out_stats, void* stream);

/*
 * Plain form: the same statistics, one window per launch sequence (each
 * window is planned and launched on its own, in order).  Same arguments and
 * results as nsgc_window_stats; kept as the per-window baseline.
 */
int nsgc_window_stats_plain(const uint32_t* src, const uint32_t* dst,
                            const int64_t* window_offsets, int64_t num_windows,
                            nsgc_stats* out_stats, void* stream);

/*
 * Process-wide switch for comparisons: with on != 0, nsgc_window_stats runs
 * the plain form (one window per launch sequence, no batching); 0 restores
 * the batched form (the default).  The graph form is not affected.  Always
 * returns NSGC_OK.  nsgc_get_plain_mode returns the current setting (0/1).
 */
int nsgc_set_plain_mode(int on);
int nsgc_get_plain_mode(void);

/*
 * Measurement form: the batched form with HIP events recorded on `stream`
 * around each phase.  Waits for the work to finish and writes the elapsed
 * milliseconds of five phases to phase_ms[0..4]: small-window kernel,
 * partition, link aggregation, row/column aggregation (with the per-window
 * combine), and the large-window tier (0 for a phase with no work).  Same
 * arguments and results as nsgc_window_stats otherwise; phase_ms is a host
 * array of 5 floats.  Not usable under stream capture.
 */
int nsgc_window_stats_timed(const uint32_t* src, const uint32_t* dst,
                            const int64_t* window_offsets, int64_t num_windows,
                            nsgc_stats* out_stats, void* stream, float* phase_ms);

/*
 * Fixed-scratch form, for callers that cannot allocate (code that must not
 * call hipMalloc, such as tight serving loops or harnesses that forbid
 * allocation).  Same arguments, results and rules as nsgc_window_stats, but
 * the plan and the workspace live in one statically sized device array per
 * GPU (NSGC_NOALLOC_SCRATCH_BYTES, of which the first NSGC_NOALLOC_PLAN_BYTES
 * hold the plan), held by each GPU the call runs on until the process ends.
 * No device memory and no pinned host memory is ever allocated; the plan is
 * staged in ordinary host memory.  The workspace needs about 24 bytes per
 * packet of the windows above 1024 packets, so batches of up to roughly
 * 5.2 million such packets fit; a batch that does not fit returns
 * NSGC_ERR_TOO_LARGE with nothing enqueued (nsgc_plan_sizes tells the plan
 * and workspace bytes of a batch beforehand).  All calls on one GPU share
 * its array, which keeps the last call's contents (each call rewrites what
 * it reads).  Overlapping calls would race on it, so the library serialises
 * them: a call on another stream than the previous call waits on the device
 * for that call to finish.  Calls on different streams therefore never run
 * concurrently in this form.  Not usable under stream capture
 * (NSGC_ERR_CAPTURING).
 */
#define NSGC_NOALLOC_SCRATCH_BYTES (128ull << 20)
#define NSGC_NOALLOC_PLAN_BYTES (2ull << 20)
int nsgc_window_stats_noalloc(const uint32_t* src, const uint32_t* dst,
                              const int64_t* window_offsets, int64_t num_windows,
                              nsgc_stats* out_stats, void* stream);

/* Human-readable text for a status code (static storage, never NULL). */
const char* nsgc_status_string(int status);

/* The hipError_t behind the last NSGC_ERR_HIP returned on this thread. */
int nsgc_last_hip_error(void);

/*
 * Pre-size the workspace pool of the current device for batches of up to
 * max_packets packets in up to max_windows windows, so that later calls
 * within those limits allocate nothing.  nsgc_reserve sizes the pool entry
 * of the null stream (the default stream of the current device);
 * nsgc_reserve_stream that of `stream` (each stream has its own entry, so
 * calls on different streams may overlap).  Waits for the stream when an
 * existing buffer has to grow.  Returns NSGC_OK, NSGC_ERR_INVALID_ARG
 * (negative sizes), NSGC_ERR_NO_MEMORY, NSGC_ERR_CAPTURING (stream being
 * captured) or NSGC_ERR_HIP.
 */
int nsgc_reserve(int64_t max_packets, int64_t max_windows);
int nsgc_reserve_stream(int64_t max_packets, int64_t max_windows, void* stream);

/* Release all workspaces of the current device (waits for the device). */
int nsgc_release(void);

/*
 * Tuning.  The planner's knobs, per window-size class (class k holds windows
 * with 2^k <= packets < 2^(k+1); class 0 also holds empty windows).
 * Every setting gives identical statistics (max_sweeps_log2 below its
 * default aside); only speed changes.
 */
typedef struct nsgc_tune_class {
  int32_t link_target;      /* packets per link bucket (sets the bucket count) */
  int32_t row_target;       /* packets per row bucket */
  int32_t col_target;       /* packets per column bucket */
  int32_t wave_target;      /* > 0: link aggregation takes one wavefront per link
                               bucket of about this many packets (64..2048), for
                               windows whose row and column bucket counts stay
                               within 256 and whose link buckets within the cap;
                               0: one workgroup per bucket of link_target packets */
} nsgc_tune_class;

typedef struct nsgc_tune {
  int32_t small_max;        /* windows with <= small_max packets run entirely in
                               LDS, one workgroup each (0..2048) */
  int32_t tile_log2;        /* partition tile: 2^tile_log2 packets (11..14) */
  int32_t link_slots_log2;  /* LDS link table: 2^k slots (10..12) */
  int32_t rc_slots_log2;    /* LDS row/column table: 2^k slots (10..13) */
  int32_t blocks_per_cu;    /* persistent grid: workgroups per compute unit (1..16;
                               each kernel is capped at what can be resident) */
  int32_t max_link_buckets_log2;  /* cap on link buckets per window (0..12) */
  int32_t max_rc_buckets_log2;    /* cap on row and on column buckets per
                                     window (0..12) */
  int32_t max_sweeps_log2;  /* a bucket whose LDS table overflows is re-run in
                               2, 4, ... sweeps; past 2^max_sweeps_log2 sweeps
                               it is abandoned and its window marked invalid
                               (0..24, default 24; lower values exist only to
                               exercise that error path) */
  int32_t combine_probes;   /* 0 (default): phase B emits one row and one
                               column entry per link.  1..64: it first combines
                               the bucket's links per source and destination
                               in LDS (one entry per id and link bucket; pays
                               off when single sources or destinations own a
                               large share of the links), with this probe
                               limit before falling back to per-link entries */
  nsgc_tune_class cls[33];
  int32_t large_min_log2;   /* windows of at least 2^k packets are computed by
                               sorting instead of hash partitioning, one window
                               at a time, with one wait for the stream each
                               (20..33; 33 turns the tier off; the graph form
                               and the entity outputs never use it) */
  int32_t row_complete;     /* 0 (default): link buckets by the hash of the whole
                               link.  1: windows whose link aggregation runs one
                               wavefront per bucket are partitioned by the
                               source hash, so that a source's links meet in
                               one bucket and that bucket yields its packets
                               and fan-out itself (stats 3-5 without a
                               phase-C pass); sources that a sample of the
                               window shows to be heavy are spread over the
                               other buckets by the destination hash, and each
                               such bucket emits one combined entry per heavy
                               source.  Not used by the entity outputs. */
} nsgc_tune;

/* Current tuning of the calling process (defaults until set). */
int nsgc_get_tune(nsgc_tune* out);
/* Validate and install a tuning; NSGC_ERR_INVALID_ARG leaves it unchanged. */
int nsgc_set_tune(const nsgc_tune* tune);
/* Built-in defaults. */
int nsgc_default_tune(nsgc_tune* out);

/*
 * Host-only planner inspection (no device work, usable without a GPU).
 * Plans num_windows windows under the current tuning and writes, per window,
 * the tier (0 = empty, 1 = small/LDS, 2 = partitioned), the log2 bucket
 * counts (link, row, column) and the number of partition tiles, plus the
 * workspace bytes the batch needs.  Any output pointer may be NULL.
 */
int nsgc_plan_inspect(const int64_t* window_offsets, int64_t num_windows,
                      int32_t* tier, int32_t* log2_link_buckets,
                      int32_t* log2_row_buckets, int32_t* log2_col_buckets,
                      int64_t* tiles, int64_t* workspace_bytes);

/*
 * Host-only sizing (no device work).  For the batch given by window_offsets,
 * under the current tuning: the bytes of its device plan and of its
 * workspace, and the upper bounds that nsgc_reserve and nsgc_graph_create
 * use for any batch of at most as many packets and windows.  The actual
 * sizes never exceed the bounds.  Any output pointer may be NULL.
 */
int nsgc_plan_sizes(const int64_t* window_offsets, int64_t num_windows, int64_t* plan_bytes,
                    int64_t* workspace_bytes, int64_t* plan_bound_bytes,
                    int64_t* workspace_bound_bytes);

/*
 * Graph form: a reusable hipGraph of the batched form with its own workspace
 * sized for up to max_packets packets and max_windows windows.  Launching
 * replays the captured graph (plan upload + persistent kernels, fixed grids);
 * only the plan's contents change between launches, so any batch within the
 * limits reuses it.  Launches of one graph object are serialised: a launch on
 * another stream than the previous one waits on the device for the previous
 * launch to finish (the two instances share one workspace).  This is the
 * form to use inside a caller's own stream capture: nsgc_graph_launch is not
 * itself capturable (it plans on the host), but its work is one graph
 * launch per call.
 */
typedef struct nsgc_graph nsgc_graph;
int nsgc_graph_create(int64_t max_packets, int64_t max_windows, nsgc_graph** out);
int nsgc_graph_launch(nsgc_graph* g, const uint32_t* src, const uint32_t* dst,
                      const int64_t* window_offsets, int64_t num_windows,
                      nsgc_stats* out_stats, void* stream);
int nsgc_graph_destroy(nsgc_graph* g);

/*
 * Per-entity outputs (Table III rows 3, 6 and 8 as vectors, and their
 * reverses; Section IV "Graph Analytics" paragraph for the globally unique
 * IP addresses).  For each window they list the non-zero entries of its
 * traffic matrix A, its sources with r(s) and f(s), its destinations with
 * c(d) and g(d), and count |{sources} U {destinations}|.  Addresses are the
 * caller's (not hashed).  Use in two steps: nsgc_window_entity_counts gives
 * each window's list lengths, the caller allocates the lists, and
 * nsgc_window_entities fills them.
 */
typedef struct nsgc_entity_counts {   /* 32 bytes per window */
  int64_t links;          /* nnz(A), = unique_links of nsgc_stats */
  int64_t sources;        /* #{s : r(s) > 0}, = unique_sources */
  int64_t destinations;   /* #{d : c(d) > 0}, = unique_destinations */
  int64_t unique_ips;     /* |{s : r(s) > 0} U {d : c(d) > 0}| */
} nsgc_entity_counts;

/*
 * The four counts per window.  Same src / dst / window_offsets / stream rules
 * as nsgc_window_stats; counts is a DEVICE array of num_windows entries,
 * fully overwritten.  Asynchronous.  Not usable under stream capture.
 */
int nsgc_window_entity_counts(const uint32_t* src, const uint32_t* dst,
                              const int64_t* window_offsets, int64_t num_windows,
                              nsgc_entity_counts* counts, void* stream);

/*
 * The lists.  links is a DEVICE array of rows of three int64 (src, dst,
 * packets = A(src, dst)); sources holds rows (s, r(s), f(s)) and
 * destinations rows (d, c(d), g(d)).  Window w writes rows
 * [link_offsets[w], link_offsets[w+1]) of links, and likewise for the other
 * two lists; the *_offsets are HOST arrays of num_windows + 1 non-decreasing
 * values >= 0 (a window's range should hold at least its count).  Rows of a
 * window come in no particular order.  counts (DEVICE, num_windows entries)
 * receives the same counts as nsgc_window_entity_counts; where a window's
 * range is shorter than its count, only that many of its rows are written
 * (which ones is unspecified) and its count still reports the full number,
 * so the caller can tell.  A list pointer may be NULL if its offsets give
 * every window an empty range.  Asynchronous.  Not usable under stream
 * capture.
 */
int nsgc_window_entities(const uint32_t* src, const uint32_t* dst,
                         const int64_t* window_offsets, int64_t num_windows,
                         const int64_t* link_offsets, int64_t* links,
                         const int64_t* source_offsets, int64_t* sources,
                         const int64_t* destination_offsets, int64_t* destinations,
                         nsgc_entity_counts* counts, void* stream);

/*
 * Address anonymization (Section IV, "IP Address Anonymization"): every
 * address of src[0..n) and dst[0..n) is replaced by a distinct integer in
 * [0, N), N the number of unique addresses of the two columns.  The paper
 * numbers the unique addresses and shuffles the numbers 0..N-1; here the
 * unique addresses are numbered in ascending order of their value and the
 * i-th maps to pi(i), pi a seeded pseudo-random permutation of [0, N): a
 * four-round Feistel network on the smallest even bit count b with
 * 2^b >= max(N, 4), round function F_r(R) = low b/2 bits of
 * mix(seed ^ (r + 1) * 0x9E3779B97F4A7C15 ^ R) for r = 0..3 (mix: the
 * SplitMix64 output function), restricted to [0, N) by cycle walking.  Equal
 * addresses get equal values in both columns, so every window's statistics
 * are unchanged.
 *
 * src, dst: DEVICE arrays of num_packets uint32 (num_packets < 2^31);
 * anon_src, anon_dst: DEVICE outputs of num_packets uint32 (they may be src
 * and dst themselves); num_addresses: DEVICE pointer to one uint64 that
 * receives N.  Asynchronous on `stream`; argument errors are reported
 * synchronously with nothing enqueued.  The workspace (about 48 bytes per
 * packet) comes from the stream's pool, as for nsgc_window_stats.  Not
 * usable under stream capture.
 */
int nsgc_anonymize(const uint32_t* src, const uint32_t* dst, int64_t num_packets, uint64_t seed,
                   uint32_t* anon_src, uint32_t* anon_dst, uint64_t* num_addresses, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NSGC_H_ */

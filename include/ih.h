/*
 * ih.h -- C ABI of libih.so: exact integral histograms on AMD MI355X (gfx950).
 *
 * The integral histogram of a uint8 frame I with H rows, W columns and B bins
 * is (Sec. 2.1, Eq. 1 of Poostchi et al., "Fast Integral Histogram
 * Computations on GPU for Real-Time Video Analytics"):
 *
 *     H(x, y, b) = #{ (x', y') : x' <= x, y' <= y, Q(I[y'][x']) == b }
 *
 * for column x in [0, W), row y in [0, H), bin b in [0, B), with the binning
 * function Q(v) = floor(v * B / 256) (the paper leaves bin edges open; these
 * are uniform bins over the 8-bit range).  Counts are exact uint32.
 *
 * Tensor layout (all entry points): H x W x B, bin index innermost,
 *     entry (x, y, b) at element offset ((size_t)y * W + x) * B + b.
 *
 * Conventions shared by every call:
 *   - Every call returns an ih_status and never aborts or throws.
 *   - Argument errors are reported before anything is launched or written.
 *   - "device" pointers are HIP device allocations on the current device;
 *     "host" pointers are ordinary host memory.  The caller owns every buffer
 *     it passes in; the library never frees caller memory.
 *   - Asynchronous calls enqueue work on the given stream and return at once;
 *     results are ready when the stream reaches that point.
 *   - A stream argument is a hipStream_t passed as void*; NULL means the
 *     null (default) stream.
 */
#ifndef IH_H_
#define IH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IH_OK = 0,
    IH_ERR_INVALID_ARG = 1,     /* null pointer, size <= 0, B outside [1,256], bad rectangle   */
    IH_ERR_RANGE = 2,           /* H*W >= 2^32: counts or indices would not fit                */
    IH_ERR_OOM = 3,             /* the library could not allocate its device scratch           */
    IH_ERR_HIP = 4,             /* a HIP runtime call failed; see ih_last_error()              */
    IH_ERR_BUDGET = 5,          /* a request exceeds the serving loop's whole HBM budget       */
    IH_NOT_READY = 6,           /* polled work has not finished yet                            */
    IH_ERR_UNKNOWN_TICKET = 7,  /* polled ticket was never issued or was already collected     */
    IH_ERR_SHUTDOWN = 8         /* the server is shutting down                                 */
} ih_status;

typedef void* ih_stream_t;      /* a hipStream_t */

/* A query rectangle with INCLUSIVE corners: columns x0..x1, rows y0..y1.
 * Valid when 0 <= x0 <= x1 < W and 0 <= y0 <= y1 < H. */
typedef struct {
    int32_t x0, y0, x1, y1;
} ih_rect;

/* A non-owning view of an integral histogram already in device memory. */
typedef struct {
    const uint32_t* data;       /* device, H*W*B uint32 in the layout above
                                   (bin-major for the *_binmajor queries)   */
    int32_t H, W, B;
    ih_stream_t stream;         /* stream the query work is enqueued on      */
} ih_view;

/*
 * ih_compute -- the integral histogram of one frame (Sec. 2.1 Eq. 1; the
 * sequential recursion of Sec. 2.2 Algorithm 1 gives the same result).
 *
 *   frame  device, H*W uint8, row-major (I[y][x] at y*W + x), read only.
 *   H, W   rows and columns, each >= 1, with H*W < 2^32.
 *   B      number of bins, 1..256.
 *   out    device, >= H*W*B uint32, written completely (layout above).
 *   stream enqueue on this stream.
 *
 * The library keeps a device scratch buffer per stream for its carries
 * (about (1/TX + 1/TY) of the output size for the chosen tile); it grows on
 * demand (the first call at a larger size synchronizes that stream) and is
 * released at process exit.  Errors: IH_ERR_INVALID_ARG, IH_ERR_RANGE,
 * IH_ERR_OOM, IH_ERR_HIP.
 */
ih_status ih_compute(const uint8_t* frame, int32_t H, int32_t W, int32_t B,
                     uint32_t* out, ih_stream_t stream);

/*
 * ih_compute_binmajor -- as ih_compute, with the result in the paper's
 * bin-major layout b x h x w (Sec. 3.1, Fig. 2): entry (x, y, b) at
 * out[(b*H + y)*W + x], so every bin is one contiguous H x W plane.  Same
 * arguments, errors and scratch as ih_compute.  ih_query reads the
 * H x W x B layout only; ih_query_binmajor reads this one.
 */
ih_status ih_compute_binmajor(const uint8_t* frame, int32_t H, int32_t W, int32_t B, uint32_t* out,
                              ih_stream_t stream);

/*
 * ih_compute_lut -- as ih_compute, with the bins given by a table: the pixel
 * of value v counts in bin lut_host[v].  The paper states the binning only as
 * membership of a pixel value in a bin (Sec. 2.1, the Q of Eq. 1); a table
 * gives bins of arbitrary edges, or any other membership (a bin may hold
 * values from several ranges, or none).  lut_host: 256 host bytes, each below
 * B.  A non-decreasing table (every bin one range of values) takes a range
 * test per bin; any other table bins each pixel through the table first.
 * The table is copied before the call returns (the caller may reuse it at
 * once); the kernels are asynchronous on stream.  Errors: as ih_compute, and
 * IH_ERR_INVALID_ARG for a null table or an entry >= B (checked before
 * anything is launched).
 */
ih_status ih_compute_lut(const uint8_t* frame, int32_t H, int32_t W, int32_t B, const uint8_t* lut_host,
                         uint32_t* out, ih_stream_t stream);

/*
 * ih_compute_noalloc -- ih_compute for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, tile choice, kernels and result as
 * ih_compute; the call itself allocates nothing (no hipMalloc, no hipFree,
 * no allocating library routine).
 *
 * The carries live in a fixed array of IH_NOALLOC_SCRATCH_BYTES inside the
 * library, one per GPU, held from the first call on that GPU until the
 * process ends.  Every call on a GPU shares that GPU's array and leaves its
 * carries in it: calls on one GPU whose work overlaps (different streams
 * without ordering between them, or several host threads) race and give
 * undefined results; calls ordered on one stream are safe.
 *
 * Errors: as ih_compute, and IH_ERR_RANGE (nothing launched) when the
 * frame's carries exceed the array.  Every frame of at most 3840 x 2160
 * pixels fits at B <= 128, and every frame of at most 7680 x 4320 pixels at
 * B <= 32; beyond that it depends on the tile ih_compute picks (1920 x 1080
 * at B = 256 and 7680 x 4320 at B = 64 fit, 3840 x 2160 at B = 256 and
 * 7680 x 4320 at B = 128 do not).
 */
#define IH_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
ih_status ih_compute_noalloc(const uint8_t* frame, int32_t H, int32_t W, int32_t B, uint32_t* out,
                             ih_stream_t stream);

/*
 * ih_query -- region histograms by the four-corner rule (Sec. 2.1, Eq. 2):
 *
 *   h(R, b) = H(x1, y1, b) - H(x0-1, y1, b) - H(x1, y0-1, b) + H(x0-1, y0-1, b)
 *
 * with H = 0 at index -1, in modular uint32 arithmetic (exact, since the
 * true count fits).
 *
 *   ih      view of a computed integral histogram (device data).
 *   rects   HOST array of n rectangles; every one is validated before
 *           anything is launched (IH_ERR_INVALID_ARG names none written).
 *           The array is copied before the call returns.
 *   n       number of rectangles; 0 is a no-op.
 *   hists   device, n*B uint32; rectangle r's histogram at r*B .. r*B+B-1,
 *           written asynchronously on ih->stream.
 */
ih_status ih_query(const ih_view* ih, const ih_rect* rects, size_t n, uint32_t* hists);

/*
 * ih_query_device -- as ih_query (Eq. 2), with the rectangles already in
 * device memory.  Each rectangle is checked on the device: an invalid one
 * gets an all-zero histogram and increments *bad_count (device uint32,
 * accumulated, not cleared by the call; may be NULL to skip counting).
 */
ih_status ih_query_device(const ih_view* ih, const ih_rect* rects_dev, size_t n,
                          uint32_t* hists, uint32_t* bad_count);

/*
 * ih_query_binmajor, ih_query_binmajor_device -- as ih_query and
 * ih_query_device (Eq. 2), on an integral histogram in the bin-major layout
 * of ih_compute_binmajor: ih->data holds B planes of H x W uint32, entry
 * (x, y, b) at (b*H + y)*W + x.  Rectangles, validation, errors, the result
 * layout (hists[r*B + b]) and the stream are those of the H x W x B calls.
 * Each bin's four corners lie in its own plane, so a rectangle costs 4*B
 * scattered reads instead of four runs of B contiguous values.
 */
ih_status ih_query_binmajor(const ih_view* ih, const ih_rect* rects, size_t n, uint32_t* hists);
ih_status ih_query_binmajor_device(const ih_view* ih, const ih_rect* rects_dev, size_t n,
                                   uint32_t* hists, uint32_t* bad_count);

/* ---------------------------------------------------------------------------
 * Batched form: many frames of uneven size and bin count, one launch per
 * phase for all of them, captured once in a hipGraph and replayed.
 * ------------------------------------------------------------------------- */

/* One frame of a batch: device pointers owned by the caller, which must stay
 * valid (and keep their addresses) for the life of the plan. */
typedef struct {
    const uint8_t* frame;       /* device, H*W uint8, row-major              */
    uint32_t* out;              /* device, H*W*B uint32 (layout above)        */
    int32_t H, W, B;
    const uint8_t* lut;         /* host, NULL for the uniform bins, else a bin
                                   table as for ih_compute_lut (256 entries,
                                   each < B), copied when the plan is
                                   created; such frames take tiles at most
                                   64 wide and are not autotuned             */
    int32_t binmajor;           /* 0: out in H x W x B; 1: out in the bin-major
                                   b x h x w layout of ih_compute_binmajor
                                   (uniform bins only: lut must be NULL; such
                                   frames take 64-column tiles with bands
                                   chosen over all of them, whatever the
                                   options force, and are not autotuned)      */
} ih_frame_desc;

typedef struct {
    int32_t autotune;       /* 1: time candidate tiles per (H, W, B) class on the
                               plan's own buffers at creation (results cached per
                               process and, if IH_AUTOTUNE_CACHE names a file, on
                               disk); 0: built-in heuristic                         */
    int32_t use_graph;      /* 1: capture the launches in hipGraphs (default)        */
    int32_t tile_x, tile_y; /* both > 0: force this tile on every frame; tile_x is
                               32 for any B, 64 for B <= 128, 128 for B == 64;
                               1 <= tile_y <= 65535 (else IH_ERR_INVALID_ARG).
                               Bin-major frames keep 64-column tiles and take
                               tile_y only                                        */
    int32_t nontemporal;    /* -1: as chosen; 0: regular stores; 1: non-temporal     */
    int64_t group_bytes;    /* > 0: pipelining.  Frames (in the order given) are
                               split into groups of about this many output bytes
                               (at least two groups, at most one per frame); a
                               group's carries are computed on a second stream
                               while the previous group's tile pass runs, so the
                               tile pass finds them in cache.  <= 0: one group,
                               all phases in order (default)                     */
    int32_t carry_bands;    /* carry schedule.  -1: as chosen (heuristic, or
                               autotuned per class); 0: reduce-then-scan (a count
                               launch, a scan launch, the tile pass); K >= 1:
                               fused -- the count launch counts bands of K tile
                               bands and scans the carries itself, so the tile
                               pass follows it directly (K is clamped to a frame's
                               band count); -2: prefix counts -- each tile block
                               of the count launch counts all rows above its
                               band (the top carries, no scan) and the tile pass
                               adds up the tile-column totals to its left (count
                               work grows with the square of the band count).
                               Frames whose geometry cannot take the schedule
                               asked for, and bin-major frames, keep
                               reduce-then-scan.                                 */
    int32_t tile_branches;  /* 0: as chosen (four); 1: the tile-pass launches (one per
                               compiled kernel variant) run one after another;
                               2..4: they are spread over that many graph
                               branches (streams) that fork after the carry
                               phases and join before the launch ends, so one
                               variant's tail overlaps another's start.  Not
                               for pipelined plans (ignored there)            */
} ih_batch_options;

/* The schedule a plan chose for one frame. */
typedef struct {
    int32_t tile_x, tile_y;     /* tile: columns x rows                             */
    int32_t nontemporal;        /* 1: non-temporal output stores                    */
    int32_t carry_bands;        /* 0: reduce-then-scan; K >= 1: fused, K tile bands
                                   per carry band; -2: prefix counts                */
    int32_t group;              /* pipeline group of the frame (0 when one group)   */
} ih_frame_schedule;

typedef struct ih_batch_plan ih_batch_plan;

typedef struct {
    int64_t frames;          /* frames in the plan                                  */
    int64_t entries;         /* sum of H*W*B                                        */
    int32_t kernel_launches; /* kernels per plan launch (all phases)                */
    int32_t tile_launches;   /* of which tile-pass kernels (one per kernel variant) */
    int32_t graph;           /* 1 if replayed from a hipGraph                        */
    int32_t groups;          /* pipeline groups (1: not pipelined)                  */
} ih_batch_info;

/*
 * ih_batch_plan_create -- plan the integral histograms (Sec. 2.1 Eq. 1) of n
 * frames.  Validates every descriptor (same rules as ih_compute), picks a tile
 * per frame (autotuned, forced or heuristic), allocates the plan's device
 * scratch (about (1/TX + 1/TY) of the total output) and job tables, and
 * captures the launches.  Autotuning runs candidate launches on `stream`,
 * writing the frames' outputs, and synchronizes it.  opt may be NULL
 * (defaults: no autotune, graph on, heuristic tiles, one group).
 * Errors: IH_ERR_INVALID_ARG, IH_ERR_RANGE, IH_ERR_OOM, IH_ERR_HIP.
 */
ih_status ih_batch_plan_create(const ih_frame_desc* frames, size_t n, const ih_batch_options* opt,
                               ih_stream_t stream, ih_batch_plan** plan);

/* Enqueue every frame's integral histogram on `stream` (one graph launch; one
 * per phase, or direct launches for a pipelined plan, while ih_profile_enable
 * is on).  A pipelined plan also runs work on a stream of its own, ordered
 * after everything enqueued on `stream` before the call; everything the call
 * enqueues completes before later work on `stream`.  Plans may be launched
 * repeatedly; launches of one plan on different streams must not overlap. */
ih_status ih_batch_plan_launch(ih_batch_plan* plan, ih_stream_t stream);

/* Waits for the plan's last launch and for its creation stream (nothing
 * else), then frees the plan's scratch, tables and graphs. */
ih_status ih_batch_plan_destroy(ih_batch_plan* plan);

ih_status ih_batch_plan_info(const ih_batch_plan* plan, ih_batch_info* info);

/* The tile chosen for frame k of the plan. */
ih_status ih_batch_plan_frame_tile(const ih_batch_plan* plan, size_t k, int32_t* tile_x,
                                   int32_t* tile_y, int32_t* nontemporal);

/* The whole schedule chosen for frame k of the plan: tile, store flavour,
 * carry schedule and pipeline group (Sec. 3.5 weighs carry schedules for the
 * tiled scans; these are this library's). */
ih_status ih_batch_plan_frame_schedule(const ih_batch_plan* plan, size_t k, ih_frame_schedule* sched);

/* ---------------------------------------------------------------------------
 * Host-transfer pipeline (Sec. 4.4, Algorithm 6): frames in host memory, whole
 * integral histograms back to host memory, copies and kernels of consecutive
 * frames overlapped on several streams.
 * ------------------------------------------------------------------------- */

typedef struct {
    double wall_ms;        /* first upload start to last download end             */
    double frames_per_s;   /* frames / wall                                        */
    double h2d_ms;         /* per-stage sums over frames, each stage timed on its  */
    double kernel_ms;      /* own stream (uploads and kernels on one, downloads on */
    double d2h_ms;         /* the other)                                           */
} ih_pipeline_stats;

/*
 * ih_transfer_pipeline -- for k in [0, n): upload frames_host[k] (H*W uint8),
 * compute its integral histogram (Sec. 2.1 Eq. 1; same kernels and tile as
 * ih_compute) and download all H*W*B uint32 of it to outs_host[k].  The
 * device holds n_streams buffer slots (1..8; 2 is the paper's double
 * buffering); frame k uses slot k mod n_streams.  Uploads and kernels run in
 * frame order on one stream, downloads in frame order on another, so one
 * frame's download overlaps the next frames' uploads and kernels while the
 * device-to-host link carries one download at a time; a slot is reused once
 * its previous frame's download has finished.  Host buffers are the caller's;
 * pinned ones (hipHostMalloc) move at full link speed, pageable ones are
 * staged by the runtime.  Output buffers must not alias.  Blocking: returns
 * when every output is in host memory; device buffers and streams are
 * allocated and freed by the call.  stats may be NULL (then no timing events
 * are recorded).
 * Errors: IH_ERR_INVALID_ARG (null pointer, n == 0, bad shape or n_streams),
 * IH_ERR_RANGE, IH_ERR_OOM, IH_ERR_HIP.
 */
ih_status ih_transfer_pipeline(const uint8_t* const* frames_host, uint32_t* const* outs_host, size_t n,
                               int32_t H, int32_t W, int32_t B, int32_t n_streams,
                               ih_pipeline_stats* stats);

/* ---------------------------------------------------------------------------
 * Served form: frame + region-query requests from many video streams.
 * ------------------------------------------------------------------------- */

typedef struct {
    uint64_t hbm_budget_bytes;  /* device memory the server may hold: resident integral
                                   histograms, uploaded frames, rectangles, results and
                                   carries (reserved as one allocation on first use)      */
    int32_t max_slots;          /* requests admitted and not yet finished, at most        */
    int32_t n_hip_streams;      /* HIP streams the work is spread over (1..16)            */
    int32_t max_batch;          /* frames per dispatched batch, at most                   */
    int32_t retain;             /* 1: keep each video stream's latest integral histogram
                                   resident (evicted oldest-first when memory is needed)  */
    uint64_t pinned_bytes;      /* pinned host staging for frames, rectangles and results,
                                   allocated on first submit (0: 1 GiB); requests that do
                                   not fit it use separately allocated pinned buffers      */
} ih_server_config;

typedef struct {
    uint64_t t_submit_ns;       /* ih_submit entered                                       */
    uint64_t t_admit_ns;        /* device memory reserved, request joined a batch           */
    uint64_t t_done_ns;         /* results in host memory, seen by the scheduler            */
} ih_timing;                    /* steady-clock nanoseconds                                 */

typedef struct ih_server ih_server;

typedef struct {
    int64_t pending;            /* submitted, waiting for admission                        */
    int64_t admitted;           /* admitted, not yet finished                              */
    int64_t retained;           /* resident integral histograms kept for later queries     */
    uint64_t device_bytes_used; /* of the budget, now                                      */
    uint64_t device_bytes_peak; /* of the budget, highest so far                           */
    uint64_t budget_blocked;    /* times the head request waited for device memory         */
} ih_server_counters;

/*
 * ih_server_create -- start a serving loop (a scheduler thread; device memory
 * and streams are set up on the first request, on the device current here).
 * Requests are admitted first-in first-out while the budget and slots allow;
 * requests that arrive while others run join the next batch as a stream frees
 * up (continuous batching), and batches on different streams overlap.
 */
ih_status ih_server_create(const ih_server_config* cfg, ih_server** server);

/*
 * ih_submit -- queue one frame (HOST memory, H*W uint8) of video stream
 * `stream_id` and nq rectangles (HOST) to answer on it by Eq. 2.  Both arrays
 * are copied before the call returns.  Returns a ticket for ih_poll.
 * Errors: IH_ERR_INVALID_ARG (shape, rectangle), IH_ERR_RANGE, IH_ERR_BUDGET
 * (the request alone exceeds the whole budget; smaller requests wait instead),
 * IH_ERR_SHUTDOWN, IH_ERR_OOM (pinned host staging).
 */
ih_status ih_submit(ih_server* server, int32_t stream_id, const uint8_t* frame_host, int32_t H, int32_t W,
                    int32_t B, const ih_rect* rects_host, size_t nq, uint64_t* ticket);

/*
 * ih_submit_lut -- as ih_submit, with each pixel value v counted in bin
 * lut_host[v] instead of Q(v) (the bin test of Eq. 1 as a table; HOST, 256
 * entries, each below B, copied before the call returns).
 * Requests with and without tables share batches.  Errors: those of
 * ih_submit, and IH_ERR_INVALID_ARG for a null or invalid table.
 */
ih_status ih_submit_lut(ih_server* server, int32_t stream_id, const uint8_t* frame_host, int32_t H, int32_t W,
                        int32_t B, const uint8_t* lut_host, const ih_rect* rects_host, size_t nq,
                        uint64_t* ticket);

/*
 * ih_poll -- IH_NOT_READY until the request has finished; then copies its
 * nq*B histograms to hists_host (HOST, may be NULL), fills *t (may be NULL),
 * forgets the ticket and returns the request's status.  Unknown or already
 * collected tickets give IH_ERR_UNKNOWN_TICKET.
 */
ih_status ih_poll(ih_server* server, uint64_t ticket, uint32_t* hists_host, ih_timing* t);

/* Eq. 2 queries on the latest resident integral histogram of a video stream
 * (servers created with retain = 1); blocks until the results are in
 * hists_host.  *frame_ticket (may be NULL) names the frame it belongs to. */
ih_status ih_server_query_latest(ih_server* server, int32_t stream_id, const ih_rect* rects_host,
                                 size_t nq, uint32_t* hists_host, uint64_t* frame_ticket);

ih_status ih_server_stats(ih_server* server, ih_server_counters* counters);

/* hold = 1: keep queueing requests but admit none (e.g. to drain the device
 * or to collect a burst); hold = 0: resume admission. */
ih_status ih_server_hold(ih_server* server, int32_t hold);

/* Stops admitting, fails still-pending requests with IH_ERR_SHUTDOWN, waits
 * for running batches, frees everything. */
ih_status ih_server_destroy(ih_server* server);

/*
 * Per-phase timing, for measurement.  While enabled, ih_compute and
 * ih_batch_plan_launch record HIP events on their stream around each of the
 * three phases (per-tile counts, carry scans, tile pass); ih_profile_read
 * waits for the recorded work and
 * returns the summed event durations.  ih_profile_enable(on) clears the
 * totals; on = 0 stops recording.  Process-wide; adds a few microseconds of
 * event records per frame while on.
 */
typedef struct {
    double agg_ms;      /* count phase: row carries and per-tile counts */
    double scan_ms;     /* carry scans                                  */
    double tile_ms;     /* tile pass: binning, scans, output stores     */
    uint64_t frames;    /* frames recorded since ih_profile_enable      */
} ih_phase_times;

ih_status ih_profile_enable(int on);
ih_status ih_profile_read(ih_phase_times* t);

/*
 * ih_write_reference -- for measurement only: writes an H x W x B uint32
 * tensor (device, layout above; each entry gets its row index) with the
 * tile pass's work items, lanes and store order for a tile_x x tile_y tile,
 * but no loads and no arithmetic.  The time it takes is what the device's
 * write path allows the tile pass in that geometry.  B <= 64; tile_x in
 * {32, 64, 128}; tile_y >= 1.  Asynchronous on stream.
 * Errors: IH_ERR_INVALID_ARG, IH_ERR_RANGE, IH_ERR_HIP.
 */
ih_status ih_write_reference(uint32_t* out, int32_t H, int32_t W, int32_t B, int32_t tile_x, int32_t tile_y,
                             ih_stream_t stream);

/* Human-readable name of a status code (static storage). */
const char* ih_status_str(ih_status s);

/* Text of the last error raised on the calling thread ("" if none). */
const char* ih_last_error(void);

/* Library version string. */
const char* ih_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IH_H_ */

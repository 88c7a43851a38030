/*
 * iqa.h -- C ABI of the MI355X (gfx950) tile-wise LISI / augLISI library.
 *
 * The library computes, for two N x N single-precision images x and y, the
 * image-quality-assessment (IQA) matrices of Li, Adamek & Armour, "GPU
 * Accelerated Image Quality Assessment-Based Software for Transient
 * Detection":
 *
 *   - pre-processing (Sec. 2): negative pixels count as zero.  NaN pixels are
 *     read as blank sky and count as zero too; -0 counts as +0.
 *   - the images are cut into (N/N_T)^2 tiles of N_T x N_T pixels (Sec. 2);
 *     tile t = ty*(N/N_T) + tx covers rows ty*N_T .. ty*N_T+N_T-1 and
 *     columns tx*N_T .. tx*N_T+N_T-1 of the row-major image.
 *   - per tile, with x', y' the clamped pixels (Eq. 1, Eq. 2, Sec. 1):
 *       A  = sum (x'+y') / (|x'-y'| + C1)        P  = sum (x'+y') * |x'-y'|
 *       Sx = sum x'                              Sy = sum y'
 *       lisi_t    = D * A / (max(Sx, Sy) + C2)                       Eq. (1)
 *       auglisi_t = 1 - P / (Sx + Sy + C)                            Eq. (2)
 *
 * Every entry point reads both images exactly once from device memory.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 * Memory.  x, y and every output are DEVICE pointers owned by the caller, on
 *   the device that is current on the calling host thread.  Images are dense,
 *   row-major (column index fastest), N*N floats each.  Inputs are read-only.
 *   Inputs and outputs must not overlap.  IQA matrices are row-major
 *   (N/N_T) x (N/N_T) floats; `sums` holds 4 floats per tile in tile order:
 *   A, P, Sx, Sy.
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the legacy
 *   default stream).  Work is enqueued on it and the call returns without
 *   waiting; results are valid once the caller synchronises that stream.
 *   Calls on the same stream are ordered; calls on different streams may run
 *   concurrently.
 * Scratch.  Shapes with few, large tiles split a tile's rows over several
 *   workgroups; each stores its partial sums, which are then added in a
 *   fixed order: by the last of them to finish, within the launch (a ticket
 *   counter decides which is last; nothing waits), when the launch has at
 *   most 1024 workgroups, else by a second, small launch on the same stream.
 *   The two give the same bits.  Those launches use a small library-owned
 *   device workspace per (device, stream) (16 bytes per tile and split part,
 *   plus 4 bytes per tile group),
 *   allocated and cleared on first use and reused afterwards (an outgrown
 *   buffer is kept until the process ends, so graphs captured earlier stay
 *   valid).  The first call for a given (device, stream, shape) must
 *   therefore not happen while the stream is being captured into a graph:
 *   call iqa_prepare() (or the entry point itself) once before.
 * Threads.  Every entry point may be called from several host threads at
 *   once, on the same stream or on different ones.  Calls on one stream run
 *   in the order they were enqueued, each launch finishing before the next
 *   starts, and a split call's two launches are enqueued back to back, so
 *   split launches on one stream share its workspace safely.  A
 *   HIP graph that captured a split-shape launch keeps the capture stream's
 *   workspace: replay it on that stream (or on one stream at a time, with
 *   nothing else using that workspace meanwhile), because two split launches
 *   running at the same time on one workspace would mix their partial sums.
 * Errors.  Every entry point validates its arguments before touching the GPU
 *   and returns a status; nothing is launched when the status is not IQA_OK.
 *   Launch failures are reported as IQA_ERR_HIP, with the HIP error code
 *   available from iqa_last_hip_error() on the same host thread.  No entry
 *   point aborts or throws.
 * Preconditions that are not checked: pixels are finite or NaN (not +-Inf) and
 *   of magnitude at most 2^50, so that the per-tile sums stay finite in FP32.
 * Precision.  Per-pixel terms are FP32; tile sums are Kahan-compensated FP32;
 *   augLISI is finalised in double-float arithmetic; the final quotients are
 *   within one unit in the last place.  Worst-case error against exact
 *   arithmetic: about 3.6e-6 (61 units of FP32 roundoff) relative to the
 *   value for the sums and LISI, and relative to max(|augLISI|,
 *   P/(Sx+Sy+C)) for augLISI; measured: below 6e-7.  Results are bitwise
 *   reproducible run to run for a given launch configuration (no floating-point
 *   atomics) and bitwise symmetric under swapping x and y.
 */
#ifndef IQA_H
#define IQA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum iqa_status {
    IQA_OK = 0,
    IQA_ERR_NULL = 1,    /* a required pointer is NULL, or no output requested */
    IQA_ERR_SHAPE = 2,   /* N or N_T not positive, N % N_T != 0, or N too large */
    IQA_ERR_ALIGN = 3,   /* a float pointer is not 4-byte aligned (sums: 16-byte) */
    IQA_ERR_PARAM = 4,   /* D, C1, C2 or C is not a positive, finite, normal float */
    IQA_ERR_HIP = 5,     /* a HIP runtime call or kernel launch failed */
    IQA_ERR_CONFIG = 6,  /* a launch configuration is invalid for the shape, or the
                            shape needs more than 2^31-1 workgroups */
    IQA_ERR_CAPTURE = 7, /* workspace would have to grow while the stream is captured */
    IQA_ERR_BUDGET = 8,  /* a request can never fit the server's HBM budget or arena */
    IQA_ERR_TIMEOUT = 9, /* a server wait ran out of time */
    IQA_ERR_SCRATCH = 10 /* the shape needs more split scratch than iqa_tiles_noalloc holds */
} iqa_status;

/* Largest supported image side: 2^17 pixels (64 GiB per FP32 image). */
#define IQA_MAX_N ((int64_t)1 << 17)

/* ------------------------------------------------------------------------ */
/* Single image pair                                                         */
/* ------------------------------------------------------------------------ */

/* Fused LISI + augLISI over every tile (Eq. 1 and Eq. 2 per tile, after the
 * clamp of Sec. 2), reading x and y once.
 *   x, y      device, N*N floats each, row-major.
 *   N, NT     image side and tile side; N % NT == 0, 1 <= N <= IQA_MAX_N.
 *   D, C1, C2 LISI constants (Eq. 1); C the augLISI constant (Eq. 2); each a
 *             positive, finite, normal float (the paper asks C1, C2, C << 1;
 *             D = C1/2 makes LISI(x, x) = S/(S + C2) ~ 1).
 *   lisi      device, (N/NT)^2 floats, or NULL to skip.
 *   auglisi   device, (N/NT)^2 floats, or NULL to skip.
 *   sums      device, 4*(N/NT)^2 floats (A, P, Sx, Sy per tile), 16-byte
 *             aligned, or NULL.
 *   stream    hipStream_t.
 * At least one of lisi, auglisi, sums must be non-NULL. */
iqa_status iqa_tiles(const float *x, const float *y, int64_t N, int64_t NT,
                     float D, float C1, float C2, float C,
                     float *lisi, float *auglisi, float *sums, void *stream);

/* LISI only (Eq. 1 per tile).  Same conventions as iqa_tiles; the values are
 * bitwise identical to iqa_tiles' lisi output. */
iqa_status lisi_tiles(const float *x, const float *y, int64_t N, int64_t NT,
                      float D, float C1, float C2, float *lisi, void *stream);

/* augLISI only (Eq. 2 per tile).  Same conventions as iqa_tiles; the values
 * are bitwise identical to iqa_tiles' auglisi output. */
iqa_status auglisi_tiles(const float *x, const float *y, int64_t N, int64_t NT,
                         float C, float *auglisi, void *stream);

/* ------------------------------------------------------------------------ */
/* Launch configuration (for the autotuner and for reproducible benchmarks)  */
/* ------------------------------------------------------------------------ */

/* How one launch maps the tiles onto the GPU.  A wave of 64 lanes is cut into
 * groups of seg*rp lanes, one group per tile: `seg` lanes stream along a tile
 * row in `vec`-float loads and `rp` such segments take interleaved rows, so a
 * wave covers ht = 64/(seg*rp) adjacent tiles and reduces them without LDS.
 * A workgroup of `waves` waves splits those tiles' rows into contiguous
 * slices (combined in LDS); `ksplit` workgroups split them further (their
 * partial sums are added by the last of them to finish, or by a second
 * launch for launches of more than 1024 workgroups).  `unroll` rows per lane are loaded
 * while the previous `unroll` are reduced. */
typedef struct iqa_launch_cfg {
    int32_t vec;     /* floats per lane load: 4, 2 or 1; NT % vec == 0 */
    int32_t waves;   /* waves per workgroup: 1, 2, 4, 8 or 16 (vec 4); 1 or 4 (vec 1, 2) */
    int32_t unroll;  /* rows per load batch: 4 or 8 (vec 4, waves <= 8); 4 otherwise */
    int32_t seg;     /* lanes per tile row segment: power of two, 1..64 */
    int32_t rp;      /* row phases per tile in a wave: power of two, seg*rp <= 64 */
    int32_t ksplit;  /* workgroups per tile group: >= 1; NT % (waves*ksplit) == 0 */
} iqa_launch_cfg;

/* The configuration iqa_tiles uses for (N, NT) and the given image pointers
 * (the pointers only matter through their alignment).  Returns IQA_ERR_SHAPE
 * for shapes iqa_tiles would reject. */
iqa_status iqa_default_cfg(int64_t N, int64_t NT, const float *x, const float *y,
                           iqa_launch_cfg *cfg);

/* Check an explicit configuration against a shape: IQA_OK or IQA_ERR_CONFIG. */
iqa_status iqa_check_cfg(int64_t N, int64_t NT, const iqa_launch_cfg *cfg);

/* iqa_tiles with an explicit launch configuration (NULL = default).  Results
 * for a given configuration are bitwise reproducible; different
 * configurations sum in different orders and agree to rounding. */
iqa_status iqa_tiles_cfg(const float *x, const float *y, int64_t N, int64_t NT,
                         float D, float C1, float C2, float C,
                         float *lisi, float *auglisi, float *sums,
                         const iqa_launch_cfg *cfg, void *stream);

/* Workgroups of the single-pair launch for (N, NT) with `cfg` (one per tile
 * group and split part); -1 if the shape or configuration is invalid. */
int64_t iqa_launch_workgroups(int64_t N, int64_t NT, const iqa_launch_cfg *cfg);

/* Split scratch held by iqa_tiles_noalloc, per GPU: 1 MiB. */
#define IQA_NOALLOC_SCRATCH_BYTES ((int64_t)1 << 20)

/* iqa_tiles_cfg for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * It calls no hipMalloc, hipFree or other allocating routine.  Split shapes
 * (cfg->ksplit > 1, or a default configuration that splits) take their
 * partial sums and ticket counters from a fixed array of
 * IQA_NOALLOC_SCRATCH_BYTES in device memory that the library holds on every
 * GPU it runs on until the process ends, instead of the per-stream workspace:
 * 4 bytes per tile group in its first 64 KiB (at most 16384 tile groups) and
 * 16 bytes per tile and split part in the rest, so a shape needing more
 * returns IQA_ERR_SCRATCH (launching nothing).  Shapes that do
 * not split use no scratch.  Results are bitwise those of iqa_tiles_cfg with
 * the same configuration.  Every call on one GPU shares that GPU's array:
 * split calls whose launches overlap in time on one GPU (different streams,
 * or graph replays running concurrently) race and must be avoided; calls
 * ordered on one stream, from any number of host threads, are safe.  The first call on a device looks up the
 * array's address (hipGetSymbolAddress) with that device current. */
iqa_status iqa_tiles_noalloc(const float *x, const float *y, int64_t N, int64_t NT,
                             float D, float C1, float C2, float C,
                             float *lisi, float *auglisi, float *sums,
                             const iqa_launch_cfg *cfg, void *stream);

/* Allocate, ahead of time, the workspace that (N, NT) with `cfg` (NULL =
 * default) needs on `stream`, so that later calls allocate nothing (e.g.
 * under graph capture).  IQA_OK when nothing or everything was allocated. */
iqa_status iqa_prepare(int64_t N, int64_t NT, const iqa_launch_cfg *cfg, void *stream);

/* ------------------------------------------------------------------------ */
/* Hierarchical aggregation (Eq. 3, Eq. 4)                                   */
/* ------------------------------------------------------------------------ */

/* Merge f x f blocks of tiles into larger tiles (Sec. 3: the IQA values of
 * tiles aggregate exactly into the value of the whole image, or of a larger
 * tile formed by merging smaller ones; Eq. 3 for LISI, Eq. 4 for augLISI).
 *   sums_in   device, ns*ns*4 floats: the `sums` output of iqa_tiles (A, P,
 *             Sx, Sy per tile, row-major tiles), 16-byte aligned.
 *   ns, f     tiles per side of the input level; f divides ns.  The output
 *             level has (ns/f)^2 tiles; f == ns gives the whole image.
 *   D, C2, C  as in iqa_tiles (C1 is already inside A).
 *   lisi, auglisi, sums_out  device, (ns/f)^2 floats / (ns/f)^2 * 4 floats,
 *             each nullable, at least one non-NULL.  sums_out feeds the next
 *             level, so a pyramid N_T, 2N_T, 4N_T, ... is a chain of calls.
 * Eq. 3/4 weight each child's index by its own denominator, which equals
 * adding the children's sums and applying Eq. 1/2 to the totals; the kernel
 * does the latter (Kahan-compensated, fixed order) and so avoids the
 * cancellation of reconstructing sums from rounded indices. */
iqa_status iqa_merge_tiles(const float *sums_in, int64_t ns, int64_t f, float D, float C2,
                           float C, float *lisi, float *auglisi, float *sums_out, void *stream);

/* ------------------------------------------------------------------------ */
/* Tuned launch shapes                                                       */
/* ------------------------------------------------------------------------ */

#define IQA_TUNE_SINGLE 0   /* shape used by iqa_tiles & co. for (N, NT) */
#define IQA_TUNE_BATCH 1    /* per-pair geometry inside iqa_tiles_batched */
#define IQA_TUNE_SERVE 2    /* per-pair geometry inside the server's batches */

/* The library's default shapes come from autotuner measurements on gfx950
 * compiled into it, falling back to a heuristic for shapes it has not seen.
 * iqa_tune_set registers a configuration for (N, NT) that takes precedence
 * over both (N == 0: for every N with this NT).  Single-pair entries are used
 * when both images are 16-byte aligned; batch entries must have vec 4,
 * ksplit 1, unroll 8 and waves 1 (one wave per tile group) or 4 (the four
 * waves of a workgroup split each tile group's rows).  IQA_ERR_CONFIG if cfg is invalid for the
 * shape.  Thread-safe; takes effect for calls made after it returns. */
iqa_status iqa_tune_set(int64_t N, int64_t NT, int kind, const iqa_launch_cfg *cfg);

/* Forget every configuration registered with iqa_tune_set (the compiled-in
 * measurements stay). */
void iqa_tune_clear(void);

/* Persistent wave count the autotuner found best for iqa_tiles_batched on
 * this GPU (2048 when no measurement is compiled in). */
int64_t iqa_batch_default_waves(void);

/* ------------------------------------------------------------------------ */
/* Ragged batches: many image pairs of mixed N and N_T in one launch         */
/* ------------------------------------------------------------------------ */

/* One image pair of a batch: the arguments of iqa_tiles for that pair. */
typedef struct iqa_pair {
    const float *x;
    const float *y;
    int64_t N;
    int64_t NT;
    float D, C1, C2, C;
    float *lisi;
    float *auglisi;
    float *sums;
} iqa_pair;

/* Bytes of one opaque per-pair batch descriptor. */
#define IQA_BATCH_DESC_BYTES 128

/* The per-pair geometry a batch uses for (N, NT) (NT % 4 == 0).  A pair's
 * batched results are bitwise equal to iqa_tiles_cfg with this config. */
iqa_status iqa_batch_cfg(int64_t N, int64_t NT, iqa_launch_cfg *cfg);

/* The per-pair geometry the server uses for (N, NT) (NT % 4 == 0): its own
 * tuned entries, chosen for the latency of a lone pair (a server's batches
 * are small), else iqa_batch_cfg's, which is chosen for the throughput of
 * large batches.  A served request's results are bitwise equal to
 * iqa_tiles_cfg with this config. */
iqa_status iqa_serve_cfg(int64_t N, int64_t NT, iqa_launch_cfg *cfg);

/* Host-side planning of a batch (no GPU calls).
 *   pairs        host array of `count` pairs; each is validated as iqa_tiles
 *                would, and must also have NT % 4 == 0 (IQA_ERR_CONFIG) and
 *                16-byte aligned images (IQA_ERR_ALIGN).
 *   descs        host buffer of count * IQA_BATCH_DESC_BYTES bytes, filled
 *                with opaque descriptors that embed the device pointers.
 *   total_units  receives the number of work units in all.  A unit is the
 *                work of one workgroup of 4 waves: four tile groups of a pair
 *                whose geometry has one wave per group, or one tile group of
 *                a pair whose geometry has four (iqa_batch_cfg says which).
 * The caller copies `descs` to device memory (16-byte aligned) unchanged and
 * passes that copy to iqa_tiles_batched; it stays valid as long as the pairs'
 * buffers do, so one copy can be launched (or graph-replayed) many times. */
iqa_status iqa_batch_describe(const iqa_pair *pairs, int64_t count, void *descs,
                              int64_t *total_units);

/* One persistent launch over every pair of a described batch.
 *   descs_dev    device copy of the descriptors from iqa_batch_describe.
 *   count, total_units  as given to / returned by iqa_batch_describe.
 *   waves        persistent waves (multiple of 4; 2048 = 8 per CU is a good
 *                start): the launch has G = min(waves/4, total_units)
 *                workgroups, and workgroup b processes units b, b+G, b+2G, ...
 * Allocates nothing and calls nothing but the launch, so it can be captured
 * into a HIP graph.  The descriptor contents are not validated on the device:
 * pass exactly what iqa_batch_describe wrote, and a device buffer that holds
 * at least `count` descriptors.  A unit number that falls outside its pair's
 * units (total_units larger than described, or count smaller) is skipped by
 * the kernel, never read from; tiles of units beyond total_units are left
 * unwritten. */
iqa_status iqa_tiles_batched(const void *descs_dev, int64_t count, int64_t total_units,
                             int64_t waves, void *stream);

/* Largest batch iqa_tiles_batched_inline takes. */
#define IQA_BATCH_INLINE_MAX 16

/* The same launch for a small batch whose descriptors stay in host memory:
 *   descs_host   host copy of the descriptors from iqa_batch_describe, for
 *                1 <= count <= IQA_BATCH_INLINE_MAX pairs (else IQA_ERR_SHAPE).
 *   total_units  must be the number iqa_batch_describe returned for exactly
 *                these descriptors: the host checks that pair i's units
 *                follow pair i-1's and that they add up (else IQA_ERR_CONFIG).
 * The descriptors travel by value in the kernel arguments, so no device table
 * and no copy precede the launch (one enqueue instead of two), and the host
 * buffer may be reused as soon as the call returns.  The argument block holds
 * 1, 4 or IQA_BATCH_INLINE_MAX descriptors, the smallest that fits `count`:
 * a launch's host-side cost grows with its argument size.  Results are bitwise
 * those of iqa_tiles_batched on the same descriptors.  Captured into a HIP
 * graph, the launch keeps the descriptors it was given. */
iqa_status iqa_tiles_batched_inline(const void *descs_host, int64_t count,
                                    int64_t total_units, int64_t waves, void *stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of snapshot-vs-reference requests            */
/* ------------------------------------------------------------------------ */

/* A server keeps reference images resident on the device and answers
 * requests "compare this snapshot with reference r at tile size NT".  A
 * scheduler thread admits requests in arrival order while the bytes held by
 * admitted, unfinished requests stay within `hbm_budget_bytes` (a request
 * holds its snapshot, 4*N*N bytes, plus its output matrices), and packs all
 * admitted requests into one batched launch (iqa_tiles_batched_inline up to
 * IQA_BATCH_INLINE_MAX requests, else iqa_tiles_batched) whenever one of
 * `streams` launch slots is free.  After each batch the slot's stream runs a
 * one-thread kernel that stores the batch's number into a word of pinned host
 * memory; the slot frees when the scheduler sees that word change (no HIP
 * event is recorded or queried per batch).  Requests arriving while batches
 * run join the next launch, so batches overlap on the device.  A request's
 * results are bitwise the same whatever it is batched with: they equal
 * iqa_tiles_cfg with the geometry of iqa_serve_cfg.  All entry points are
 * thread-safe. */
typedef struct iqa_server iqa_server;

typedef struct iqa_server_opts {
    int64_t hbm_budget_bytes;  /* admission cap, > 0 */
    int64_t host_arena_bytes;  /* per slot: device room for snapshots copied from
                                  host memory (0: device snapshots only) */
    int64_t waves;             /* persistent waves per launch; 0 = tuned default */
    int32_t streams;           /* launch slots = batches in flight, 1..16 */
    int32_t max_batch;         /* requests per launch, 1..2^20 */
    float D, C1, C2, C;        /* Eq. 1 / Eq. 2 constants for every request */
    int64_t idle_spin_ns;      /* with nothing to do, keep polling this long after
                                  the last work before sleeping (0..1e9; 0 sleeps
                                  at once; polling occupies one CPU core) */
} iqa_server_opts;

/* Ordering with the caller's own work.  The server runs each batch on its
 * own streams, which are not ordered after any stream of the caller.  A
 * snapshot or an output buffer that work on a caller's stream still writes
 * or reads (a snapshot produced by a kernel, an output buffer a caching
 * allocator just handed out) therefore needs `ready_event`: a hipEvent_t
 * recorded on that stream after that work.  The batch that carries the
 * request waits for it on the device (hipStreamWaitEvent) before it reads
 * the snapshot or writes the outputs.  The event must stay valid until the
 * request completes.  With ready_event NULL the caller guarantees that the
 * snapshot is complete and the outputs are unused when it submits (e.g. after
 * synchronising the producing stream). */
typedef struct iqa_request {
    const float *snapshot_dev;   /* device N x N snapshot (16-byte aligned), or NULL */
    const float *snapshot_host;  /* pinned host snapshot, or NULL; exactly one is set */
    float *lisi;                 /* device outputs as in iqa_tiles (at least one), */
    float *auglisi;              /* owned by the caller, untouched until the request */
    float *sums;                 /* completes */
    int64_t NT;                  /* tile side: divides the reference's N, NT % 4 == 0 */
    int32_t ref_id;              /* from iqa_server_add_reference */
    int32_t reserved;
    uint64_t tag;                /* returned in the completion */
    void *ready_event;           /* hipEvent_t the request's batch waits for, or NULL */
} iqa_request;

typedef struct iqa_completion {
    uint64_t tag;
    int32_t status;              /* IQA_OK, or why the request was rejected / failed */
    int32_t reserved;
    int64_t t_submit_ns;         /* steady-clock times: submitted, admitted, */
    int64_t t_admit_ns;          /* launched, seen complete by the scheduler, */
    int64_t t_launch_ns;         /* and handed to the caller by iqa_server_poll */
    int64_t t_done_ns;
    int64_t t_poll_ns;
} iqa_completion;

typedef struct iqa_server_stats {
    int64_t submitted, completed, rejected, batches, max_batch;
    int64_t in_flight_bytes, peak_in_flight_bytes;
    int32_t last_hip_error;
    int32_t reserved;
} iqa_server_stats;

/* Start a server (and its scheduler thread) on the current device.  Returns
 * IQA_ERR_CONFIG for out-of-range options, IQA_ERR_HIP if a stream, event or
 * buffer cannot be created. */
iqa_status iqa_server_create(const iqa_server_opts *opts, iqa_server **out);

/* Dry run, for capacity planning and for testing the scheduling policy
 * without a GPU: a server that admits, batches and retires requests exactly
 * like iqa_server_create's but launches nothing and makes no HIP call.  A
 * batch of b input bytes completes fixed_ns + b / bytes_per_ns nanoseconds
 * after its launch; outputs are not written.  Reference and snapshot pointers
 * are only checked for alignment, never dereferenced. */
iqa_status iqa_server_create_dry(const iqa_server_opts *opts, int64_t fixed_ns,
                                 double bytes_per_ns, iqa_server **out);

/* Register a resident reference (device, N x N, 16-byte aligned, owned by the
 * caller and kept alive until iqa_server_destroy).  Only before the first
 * submit. */
iqa_status iqa_server_add_reference(iqa_server *sv, const float *ref, int64_t N,
                                    int32_t *ref_id);

/* Queue `count` requests.  Invalid requests, and requests that could never
 * fit the budget (IQA_ERR_BUDGET), complete at once with that status. */
iqa_status iqa_server_submit(iqa_server *sv, const iqa_request *reqs, int64_t count);

/* Move up to `max` completions to `out` (host); returns how many.  Never
 * blocks. */
int64_t iqa_server_poll(iqa_server *sv, iqa_completion *out, int64_t max);

/* Wait until every submitted request has completed (IQA_ERR_TIMEOUT after
 * timeout_ms). */
iqa_status iqa_server_drain(iqa_server *sv, int64_t timeout_ms);

iqa_status iqa_server_get_stats(iqa_server *sv, iqa_server_stats *stats);

/* Open-loop trace replay, for measurement: a separate thread submits
 * reqs[i] at start + arrival_ns[i] (non-decreasing), whatever the state of
 * the server, while this call collects the `count` completions into `out`
 * (completion order; times relative to the start of the trace). */
iqa_status iqa_server_replay(iqa_server *sv, const iqa_request *reqs,
                             const int64_t *arrival_ns, int64_t count, iqa_completion *out,
                             int64_t timeout_ms);

/* Finish every queued request, stop the scheduler, free the server. */
iqa_status iqa_server_destroy(iqa_server *sv);

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                               */
/* ------------------------------------------------------------------------ */

/* Streaming-read reference kernel, for measurement only: `blocks`
 * workgroups of 256 threads each sum a contiguous share of the n floats at
 * `buf` (device, 16-byte aligned, n % 4 == 0) with the same non-temporal
 * 16-byte loads as the tile kernels, and write one float each to `out`
 * (device, `blocks` floats).  Its bandwidth is the attainable HBM read rate
 * that the tile kernels are compared with; the sums carry no meaning. */
iqa_status iqa_read_ceiling(const float *buf, int64_t n, float *out, int64_t blocks,
                            void *stream);

/* iqa_tiles_cfg with a per-workgroup timeline, for measuring where a launch's
 * time goes (vec 4 configurations only, else IQA_ERR_CONFIG).  The results
 * are those of iqa_tiles_cfg with the same configuration, bitwise.
 *   stamps       device, stamp_count uint64 (8-byte aligned), at least
 *                8 * iqa_launch_workgroups(N, NT, cfg) (else IQA_ERR_SHAPE).
 *                Workgroup b (in launch order) writes stamps[8b .. 8b+7]:
 *                wall-clock ticks (see hipDeviceAttributeWallClockRate) of its
 *                first wave's entry, of its first batch of rows reduced (its
 *                first loads back), of its last rows reduced (its last loads
 *                back) and of its exit once its results were stored; then the
 *                XCC_ID and HW_ID hardware registers it ran with, its tile
 *                group, and its split part with bit 32 set when this
 *                workgroup finished its tiles (always, without a split; for
 *                the part that came last, with one).
 * The stamps cost a few instructions per workgroup; the product entry points
 * are separate kernels without them. */
iqa_status iqa_tiles_timeline(const float *x, const float *y, int64_t N, int64_t NT, float D,
                              float C1, float C2, float C, float *lisi, float *auglisi,
                              float *sums, const iqa_launch_cfg *cfg, uint64_t *stamps,
                              int64_t stamp_count, void *stream);

/* Measurement probes (they compute nothing the library returns).
 * iqa_probe_empty: one launch of an empty kernel, `blocks` workgroups of
 *   `threads` (1..1024) threads: the fixed cost of a launch.
 * iqa_probe_read: a plain read of the n floats at `buf` (device, 16-byte
 *   aligned, n % 4 == 0) by `blocks` workgroups of `threads` threads (a
 *   multiple of 64, at most 1024), each summing a contiguous share with
 *   `loads` (4, 8, 16 or 32) 16-byte loads in flight per lane, and writing
 *   one float to `out` (device, `blocks` floats).  `mode`:
 *     IQA_PROBE_READ_REGS         loads into registers, kernel arguments
 *                                 preloaded into SGPRs at wave start;
 *     IQA_PROBE_READ_REGS_STRUCT  the same, arguments loaded from memory;
 *     IQA_PROBE_READ_LDS          loads straight into LDS (16 bytes per
 *                                 lane per load, loads * threads * 16 bytes
 *                                 of LDS, at most 64 KiB, else
 *                                 IQA_ERR_CONFIG).
 * iqa_probe_read_timeline: the IQA_PROBE_READ_REGS read with per-workgroup
 *   wall-clock stamps in iqa_tiles_timeline's record layout (8 uint64 per
 *   workgroup at stamps[8 * workgroup]: entry, first loads summed, last loads
 *   summed, exit after its store, XCC_ID, HW_ID, workgroup index, 1 << 32;
 *   stamp_count >= 8 * blocks, else IQA_ERR_SHAPE), so that the read floor
 *   and the tile kernel split their time the same way.
 * The HIP error behind an IQA_ERR_HIP is iqa_probe_last_hip_error(). */
#define IQA_PROBE_READ_REGS 0
#define IQA_PROBE_READ_REGS_STRUCT 1
#define IQA_PROBE_READ_LDS 2
iqa_status iqa_probe_empty(int64_t blocks, int32_t threads, void *stream);
iqa_status iqa_probe_read(const float *buf, int64_t n, float *out, int64_t blocks,
                          int32_t threads, int32_t loads, int32_t mode, void *stream);
iqa_status iqa_probe_read_timeline(const float *buf, int64_t n, float *out, int64_t blocks,
                                   int32_t threads, int32_t loads, uint64_t *stamps,
                                   int64_t stamp_count, void *stream);
int iqa_probe_last_hip_error(void);

/* Rate of the device wall clock that iqa_tiles_timeline's stamps count, in
 * kHz, for the current device (-1 if it cannot be read). */
int64_t iqa_wall_clock_khz(void);

/* Static, human-readable name of a status code. */
const char *iqa_status_str(int status);

/* The HIP error code behind the last IQA_ERR_HIP on this host thread (0 if
 * none). */
int iqa_last_hip_error(void);

/* Library ABI version: major*10000 + minor*100 + patch. */
int iqa_version(void);

#ifdef __cplusplus
}
#endif

#endif /* IQA_H */

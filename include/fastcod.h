/*
 * fastcod.h -- C-ABI of libfastcod.so: pass-through connectivity counting on MI355X (gfx950).
 *
 * The operation (FastCod, Bian et al., SPIE Medical Imaging 2023; Section 2 "Method", Alg. 2:
 * passthrough, loc2region and the update of C; the abstract and Section 1 define two regions as
 * connected when a streamline passes through both, wherever it starts or ends):
 *
 *   A streamline l is an ordered list of points p^1..p^T in voxel coordinates (voxel centres at
 *   integers).  Each point lies in voxel ( floor(fl32(x+0.5)), floor(fl32(y+0.5)), floor(fl32(z+0.5)) )
 *   -- one IEEE binary32 add rounded to nearest even, then an exact floor; a point whose voxel is
 *   outside the grid, or with a NaN/inf coordinate, touches nothing.
 *   I_l = distinct ROI rows roi[v] in [0,N) over the voxels v of l,
 *   M_l = distinct target labels lab[v] in [0,M) over the voxels v of l,
 *   C[i][m] = number of streamlines l with i in I_l and m in M_l.
 *   With a coordinate scale s (the super-resolution transform of Section 3, "Super-resolving
 *   connectivity features"), every coordinate is first replaced by fl32(p*s).
 *
 * Conventions for every entry point:
 *   - Pointers are DEVICE pointers unless marked HOST.  The caller owns every buffer it passes;
 *     the library never frees caller memory.
 *   - Volumes are int32 [Z][Y][X], x fastest: lin = x + X*(y + Y*z).  Values outside [0,N)
 *     (ROI) or [0,M) (labels) mean "no ROI" / "no target" (-1 is the usual choice).
 *   - Streamlines: points float32 [P][3] (x,y,z interleaved); offsets int64 [S+1] with
 *     offsets[0] = 0, nondecreasing, offsets[S] = P; streamline s is points[offsets[s], offsets[s+1]).
 *     Kernels clamp every offset into [0, offsets[S]], so malformed offsets give wrong counts but
 *     never a read outside points[0, offsets[S]).  FASTCOD_VALIDATE checks them first.
 *   - Argument errors are detected synchronously, before anything is enqueued, and return
 *     FASTCOD_EINVAL.  HIP failures return FASTCOD_EHIP.  fastcod_last_error() gives the detail
 *     (thread-local).  No C++ exception crosses this interface.
 *   - Counting calls are asynchronous on `stream` (a hipStream_t; NULL = the null stream):
 *     results are valid once the stream is synchronised.  Calls on one stream are serialised by
 *     the stream; the library keeps a workspace per (device, stream) -- per calling thread for
 *     hipStreamPerThread, which names a different stream in every thread -- and grows it with
 *     hipMalloc on first use (that growth synchronises the device).  At most 8 workspaces are kept
 *     per device: a call on a ninth stream first frees the least recently used idle one (after a
 *     device synchronisation).  fastcod_release() frees them all.
 *   - C is int32; one call adds at most S to any entry, and S <= INT32_MAX is enforced.
 */
#ifndef FASTCOD_H
#define FASTCOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define FASTCOD_OK 0
#define FASTCOD_EINVAL (-1)    /* bad argument (null pointer, size out of range, overflow)        */
#define FASTCOD_ERANGE (-2)    /* FASTCOD_VALIDATE / fastcod_validate found malformed input data   */
#define FASTCOD_ENOMEM (-3)    /* device allocation failed, or a request exceeds a memory budget   */
#define FASTCOD_EHIP (-4)      /* a HIP runtime call failed                                        */
#define FASTCOD_EBUSY (-5)     /* the object is in use (e.g. server still has requests in flight)  */
#define FASTCOD_ECANCELED (-6) /* the request was cancelled                                        */
#define FASTCOD_ETIMEDOUT (-7) /* a wait ended before the request finished                         */

/* fastcod_opts.flags */
#define FASTCOD_ACCUMULATE 1u  /* add into C_out instead of overwriting it                         */
#define FASTCOD_VALIDATE 2u    /* run fastcod_validate first (synchronous); ERANGE if it fails      */

/* fastcod_opts.variant: which counting kernel runs (all give identical C). */
#define FASTCOD_VARIANT_AUTO 0   /* the library's choice (the flat point-stream kernel)            */
#define FASTCOD_VARIANT_WAVE 1   /* one wavefront per streamline, raster volume lookups            */
#define FASTCOD_VARIANT_STREAM 2 /* flat point stream split at streamline starts, compact volume   */

/* fastcod_opts.mode: which target labels a streamline contributes (Section 2; Alg. 1 and 2).
 * Rows are always I_l, the ROI rows the streamline passes through, except in SEED_END. */
#define FASTCOD_MODE_PASSTHROUGH 0 /* labels of every point: C(i, m) for m passed through (default)  */
#define FASTCOD_MODE_END 1         /* Alg. 2 as printed: loc2region of the last point p^T only       */
#define FASTCOD_MODE_BOTH_ENDS 2   /* labels of the first and the last point (a shared one once)     */
#define FASTCOD_MODE_SEED_END 3    /* Alg. 1's count: C(row of p^1, label of p^T) += 1 per streamline; */
                                   /* the seed is the first point                                      */

typedef struct fastcod_opts {
    float scale;        /* coordinate scale s applied before voxelisation; 1.0f = none              */
    int32_t upsample;   /* u in 1..4: u - 1 evenly spaced points inserted between neighbouring points */
                        /* before counting (Section 3, super-resolving connectivity features):     */
                        /* y = fl32(q_k + fl32(a_t * fl32(q_k+1 - q_k))), a_t = fl32(t/u), on the    */
                        /* scaled points q, no FMA; u > 1 needs FASTCOD_MODE_PASSTHROUGH; 1 = none   */
    uint32_t flags;     /* FASTCOD_ACCUMULATE | FASTCOD_VALIDATE                                    */
    int32_t variant;    /* FASTCOD_VARIANT_*                                                        */
    void *event_begin;  /* optional hipEvent_t, recorded on `stream` just before the counting kernel */
    void *event_end;    /* optional hipEvent_t, recorded on `stream` just after it                  */
    int32_t batch;      /* flat-stream schedule: 64-point windows per pipelined batch, 2 or 4; 0 = 4 for
                           n_streamlines >= 2^21 (ranges long enough to fill the deeper pipeline), else 2 */
    int32_t blocks_per_cu; /* flat-stream schedule: resident workgroups per CU, 0 = occupancy limit */
    int32_t mode;       /* FASTCOD_MODE_*; the batched and served forms count FASTCOD_MODE_PASSTHROUGH */
    int64_t pair_capacity; /* flat-stream path: workspace entries (4 bytes each, held twice) for the   */
                        /* C updates it appends and later adds into C tile by tile; 0 = 8 per       */
                        /* streamline, clamped to [2^20, 2^28]; values above INT32_MAX are clamped.  */
                        /* Updates that find their wavefront's share full go to C as atomics: the   */
                        /* result is the same, only slower.  With 0, calls of fewer than 2^17       */
                        /* streamlines on a C of at most 2^20 entries use no pair buffer and add    */
                        /* every update to C as an atomic.  Must be >= 0.                            */
} fastcod_opts;

/* Default options: {1.0f, 1, 0, FASTCOD_VARIANT_AUTO, NULL, NULL, 0, 0, FASTCOD_MODE_PASSTHROUGH, 0}. */
fastcod_opts fastcod_default_opts(void);

/*
 * Pass-through connectivity matrix (Section 2, Alg. 2), overwriting C_out.
 *   points           [P][3] float32, device
 *   offsets          [S+1] int64, device
 *   n_streamlines    S, 0 <= S <= INT32_MAX
 *   roi_index_vol    [Z][Y][X] int32, device; value in [0,N) = row of C
 *   target_label_vol [Z][Y][X] int32, device; value in [0,M) = column of C
 *   dims             HOST int32[3] = {X, Y, Z}, each >= 1, X*Y*Z < 2^31
 *   N, M             >= 1, N*M < 2^31
 *   C_out            [N][M] int32 row-major, device; overwritten
 *   stream           hipStream_t (NULL = null stream)
 * Returns FASTCOD_OK once all work is enqueued.
 */
int fastcod_count(const float *points, const int64_t *offsets, int64_t n_streamlines,
                  const int32_t *roi_index_vol, const int32_t *target_label_vol,
                  const int32_t dims[3], int32_t N, int32_t M, int32_t *C_out, void *stream);

/* Same as fastcod_count with options (NULL opts = defaults). */
int fastcod_count_ex(const float *points, const int64_t *offsets, int64_t n_streamlines,
                     const int32_t *roi_index_vol, const int32_t *target_label_vol,
                     const int32_t dims[3], int32_t N, int32_t M, int32_t *C_out,
                     const fastcod_opts *opts, void *stream);

/*
 * Resident volume: the two label volumes of one grid, preprocessed once into a compact
 * lookup structure (an occupancy bit per voxel in 16x8x8 bricks plus the packed (row, label)
 * codes of occupied voxels) that stays in device memory.  Section 2's loc2region and
 * passthrough then read a few MB instead of both volumes.  The source volumes may be freed
 * after creation.  The handle is ready for use on any stream once `stream` has completed
 * the build; counting calls made through it wait for that build automatically.
 */
typedef struct fastcod_volume fastcod_volume;

int fastcod_volume_create(const int32_t *roi_index_vol, const int32_t *target_label_vol,
                          const int32_t dims[3], int32_t N, int32_t M, void *stream,
                          fastcod_volume **out);
/* Device bytes held by the handle. */
size_t fastcod_volume_bytes(const fastcod_volume *vol);
/* Counting against a resident volume; arguments as fastcod_count_ex. */
int fastcod_volume_count(const fastcod_volume *vol, const float *points, const int64_t *offsets,
                         int64_t n_streamlines, int32_t *C_out, const fastcod_opts *opts,
                         void *stream);
/* Frees the handle (synchronises its device first). */
int fastcod_volume_destroy(fastcod_volume *vol);

/*
 * fastcod_volume_count without any device allocation, for callers that cannot allocate: code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Arguments,
 * result and asynchrony are those of fastcod_volume_count (the volume handle is created
 * beforehand; C_out and the streamlines stay the caller's).  Instead of the per-stream workspace,
 * every call on a device uses one fixed scratch area of 72 MiB that the library holds on that
 * device until the process ends; nothing is allocated or freed by the call.  Limits: at most 2^21
 * streamlines per call (EINVAL beyond), at most 2^21 appended C updates (the rest go to C as
 * atomics, same result), a C of more than 2^26 entries takes atomics into C_out itself (no
 * transposed copy), and N and M whose overflow bit maps exceed 4 MiB fail with ENOMEM -- every
 * such check happens before anything is enqueued.  Calls on one device share the area: calls
 * that overlap in time on one device (two streams, or two threads) race and give wrong counts,
 * so serialise them (one stream).  The area keeps the last call's contents; each call clears what
 * it needs zeroed with a kernel of its own (no memset node under capture).
 */
int fastcod_volume_count_noalloc(const fastcod_volume *vol, const float *points, const int64_t *offsets,
                                 int64_t n_streamlines, int32_t *C_out, const fastcod_opts *opts, void *stream);

/*
 * Batched form: many subjects (each its own streamlines, volumes, N, M, scale, mode, upsampling and
 * C) counted by persistent kernels that take (subject, point range) work items from a counter, the
 * whole sequence (zero every C, end labels, partition, count, overflow fallback, transposes) captured
 * once in a hipGraph and replayed by every launch.  Subjects of one kind share one launch: all the
 * pass-through subjects (the usual case) one, the endpoint-mode subjects (Alg. 2 as printed,
 * Section 2) another, upsampled ones (Section 3) a third, Alg. 1's seed-to-end subjects a fourth.
 * Each subject's C is identical to what fastcod_count_ex gives for it with the same scale, mode and
 * upsample (counts are exact integers and C is additive over streamline ranges).
 */
typedef struct fastcod_subject {
    const float *points;              /* [P][3] float32, device                                         */
    const int64_t *offsets;           /* [S+1] int64, device                                             */
    int64_t n_streamlines;            /* S, 0 <= S <= INT32_MAX                                          */
    const int32_t *roi_index_vol;     /* [Z][Y][X] int32, device                                         */
    const int32_t *target_label_vol;  /* [Z][Y][X] int32, device                                         */
    int32_t dims[3];                  /* {X, Y, Z}, each >= 1, X*Y*Z < 2^31                              */
    int32_t N, M;                     /* N, M >= 1, N*M < 2^31                                           */
    float scale;                      /* coordinate scale, finite and > 0 (1.0f = none)                  */
    int32_t *C_out;                   /* [N][M] int32, device; overwritten by every launch.  Subjects of
                                         one plan may share a C_out only with equal N and M: it then
                                         receives the sum of their counts                            */
    int32_t mode;                     /* FASTCOD_MODE_* of this subject (0 = pass-through)               */
    int32_t upsample;                 /* u in 1..4 as fastcod_opts.upsample (0 = 1); u > 1 needs mode 0  */
} fastcod_subject;

/* Schedule of the batched kernel (chosen by the tuner or the defaults). */
typedef struct fastcod_schedule {
    int32_t batch;           /* 64-point windows per pipelined batch: 2 or 4                             */
    int32_t blocks_per_cu;   /* resident 256-thread workgroups per CU                                    */
    int32_t items_per_wave;  /* work items per wavefront (point-balanced over all subjects)              */
    float tuned_ms;          /* duration of one launch measured by the tuner (0 if not tuned)           */
} fastcod_schedule;

typedef struct fastcod_plan fastcod_plan;

#define FASTCOD_PLAN_TUNE 1u  /* time candidate schedules on these subjects and keep the fastest        */

/*
 * Builds a plan (synchronous on `stream`): compact volumes of every distinct volume pair (built
 * once, kept by the plan; the source volumes may be freed afterwards), work-item tables, scratch,
 * and the captured graph.  A subject with streamlines, N >= 64, M >= 2 and a C_out that no other
 * subject of the plan writes is counted into a plan-owned transposed copy [M][N] (4*N*M bytes),
 * transposed into C_out at the end of each launch; the others count into C_out directly.  Points, offsets and C_out are read/written by every launch, so their
 * contents may change between launches but their addresses and sizes may not.
 * tune_cache: optional HOST path of a text file of tuned schedules (read, and appended to when
 * FASTCOD_PLAN_TUNE times a new kind of batch); NULL = no file.
 * Errors: EINVAL (bad subject, or a grid too thin for the compact volume), ENOMEM, EHIP.
 */
int fastcod_plan_create(const fastcod_subject *subjects, int32_t n, uint32_t flags, const char *tune_cache,
                        void *stream, fastcod_plan **out);
/* One replay of the captured graph on `stream` (asynchronous).  Launches of one plan must not
 * overlap in time (they share the plan's counters); serialise them on one stream. */
int fastcod_plan_launch(fastcod_plan *plan, void *stream);
/* The schedule the plan uses. */
int fastcod_plan_get_schedule(const fastcod_plan *plan, fastcod_schedule *out);
/* Frees the plan (synchronises its device first). */
int fastcod_plan_destroy(fastcod_plan *plan);
/* create + launch + synchronise + destroy, default schedule. */
int fastcod_count_batched(const fastcod_subject *subjects, int32_t n, void *stream);

/*
 * Served form: a server that keeps volume pairs resident on one device and counts requests as
 * they arrive, each request's C identical to fastcod_count_ex on the same inputs, scale, mode and
 * upsampling (C is a sum of exact per-streamline terms, Section 2, so cutting a request into
 * streamline ranges and interleaving them with other requests changes nothing).
 *
 * The server takes one device allocation of memory_budget bytes at creation and places in it the
 * compact volumes and every admitted request's device data: its offsets, its points unless they
 * are already on the device, and its C unless C_out is on the device.  Requests are admitted
 * first come, first served when their bytes (plus their volume's compact form and build scratch,
 * if the volume is not resident) fit; idle volumes are evicted least recently used first to make
 * room, and rebuilt from the server's host copy when needed again.  A request that could never
 * fit is refused at submission with FASTCOD_ENOMEM.  Admitted requests are counted by one launch
 * at a time that takes the next streamline range of every active request (about tick_points
 * points in all): about chunk_points points of each (an equal part of the launch when more are
 * active than that allows) and the rest for the oldest requests first.  A new request thus starts
 * counting at the next launch, and the oldest ones finish first.  Host points are uploaded
 * in pieces of about chunk_points points that overlap the counting.  A scheduler thread owned by
 * the server issues all device work on its own streams; the calls below only touch host state
 * and may come from any thread.
 */
typedef struct fastcod_server fastcod_server;

typedef struct fastcod_server_config {
    uint64_t memory_budget;  /* device bytes for volumes and requests; 0 = 80% of the free memory     */
    int64_t tick_points;     /* points per counting launch over all active requests; 0 = 2^27         */
    int64_t chunk_points;    /* host upload piece and smallest per-request share of a launch; 0 = 2^20 */
    int32_t max_active;      /* admitted requests still counting, 1..1024; 0 = 64 (one whose result   */
                             /* is being copied out no longer counts)                                 */
    int32_t reserved;        /* must be 0                                                              */
} fastcod_server_config;

#define FASTCOD_REQ_DEVICE_POINTS 1u  /* request.points is a device pointer (else host)             */
#define FASTCOD_REQ_DEVICE_C 2u       /* request.C_out is a device pointer (else host)              */
#define FASTCOD_REQ_AFTER_STREAM 4u   /* order every device access of the request after the work    */
                                      /* enqueued on request.stream before the submission            */

typedef struct fastcod_request {
    int32_t volume_id;         /* from fastcod_server_add_volume                                    */
    uint32_t flags;            /* FASTCOD_REQ_*                                                     */
    const float *points;       /* [P][3] float32, HOST unless FASTCOD_REQ_DEVICE_POINTS             */
    const int64_t *offsets;    /* [S+1] int64, HOST; offsets[0] = 0, nondecreasing, P = offsets[S]  */
    int64_t n_streamlines;     /* S, 0 <= S <= INT32_MAX                                            */
    float scale;               /* coordinate scale, finite and > 0 (1.0f = none)                    */
    int32_t *C_out;            /* [N][M] int32 of the volume, HOST unless FASTCOD_REQ_DEVICE_C;     */
                               /* overwritten with the result when the request finishes             */
    int32_t mode;              /* FASTCOD_MODE_* (0 = pass-through)                                 */
    int32_t upsample;          /* u in 1..4 as fastcod_opts.upsample (0 = 1); u > 1 needs mode 0    */
    void *stream;              /* with FASTCOD_REQ_AFTER_STREAM: the hipStream_t (NULL = the null   */
                               /* stream) whose work produced device-resident points or C_out       */
} fastcod_request;

typedef struct fastcod_request_info {
    int32_t status;            /* FASTCOD_OK, FASTCOD_ECANCELED, or the error that failed the server */
    int64_t t_submit_ns;       /* CLOCK_MONOTONIC times: submission, admission, result in C_out     */
    int64_t t_admit_ns;
    int64_t t_done_ns;
    int64_t chunks;            /* counting launches that took part of the request                   */
    int64_t device_bytes;      /* device bytes the request held while admitted (volume excluded)    */
} fastcod_request_info;

typedef struct fastcod_server_stats {
    uint64_t budget_bytes;     /* arena size                                                        */
    uint64_t used_bytes;       /* arena bytes in use (resident volumes + admitted requests)         */
    int64_t pending, active;   /* requests waiting for admission / admitted and unfinished          */
    int64_t completed;         /* requests finished (any status)                                    */
    int64_t launches;          /* counting launches issued                                          */
    int64_t volume_builds;     /* compact volume builds (first use and rebuilds after eviction)     */
    int64_t evictions;         /* volumes evicted to make room                                      */
    int32_t failed;            /* 0, or the error status that stopped the server                    */
    int32_t reserved;
} fastcod_server_stats;

/* Creates a server on the current device (synchronous).  NULL cfg = defaults.
 * Errors: EINVAL (bad config), ENOMEM (the budget cannot be allocated), EHIP. */
int fastcod_server_create(const fastcod_server_config *cfg, fastcod_server **out);
/* Registers a volume pair from HOST memory (int32 [Z][Y][X], copied by the server, so the caller's
 * arrays may be freed on return).  The compact form is built on the device at the first request
 * that needs it.  Errors: EINVAL (as fastcod_count_ex's volume arguments, or a grid too thin for
 * the compact volume), ENOMEM (the volume alone exceeds the budget). */
int fastcod_server_add_volume(fastcod_server *srv, const int32_t *roi_index_vol_host,
                              const int32_t *target_label_vol_host, const int32_t dims[3], int32_t N,
                              int32_t M, int32_t *volume_id);
/* Queues a request.  Its points, offsets and C_out must stay valid and unchanged until it has
 * finished (fastcod_server_wait returned its status).  Host arrays must hold their data at
 * submission.  The server's device work runs on streams of its own: for device-resident points
 * or C_out written by work still in flight on some stream, set FASTCOD_REQ_AFTER_STREAM and name
 * that stream -- an event recorded on it here orders every device access of the request after
 * that work (without the flag the caller must have completed that work before submitting).
 * Offsets: ERANGE here if offsets[0] != 0 or offsets[n_streamlines] < 0; that none decreases is
 * checked on the device when the request is set up (after admission, before it is counted), and a
 * request whose offsets decrease finishes with FASTCOD_ERANGE from fastcod_server_wait, C_out
 * untouched.  Errors: EINVAL, ERANGE, ENOMEM (can never fit the budget), EBUSY (server shutting
 * down), EHIP (the event could not be recorded on request.stream), or the status that failed the
 * server. */
int fastcod_server_submit(fastcod_server *srv, const fastcod_request *req, uint64_t *request_id);
/* Waits up to timeout_us microseconds (< 0: no limit) for a request to finish.  Returns its
 * status (FASTCOD_OK: C_out holds the result) and fills *info (may be NULL); the request's record
 * is then dropped, so each id is waited for once.  FASTCOD_ERANGE: its offsets decrease (C_out
 * untouched).  FASTCOD_ETIMEDOUT: still running (not an error of the request); FASTCOD_EINVAL:
 * unknown id. */
int fastcod_server_wait(fastcod_server *srv, uint64_t request_id, int64_t timeout_us,
                        fastcod_request_info *info);
/* Cancels a request.  A pending one finishes at once; an admitted one takes no further launches
 * and finishes with FASTCOD_ECANCELED once its issued device work has drained (C_out is then
 * unspecified; one whose result copy was already issued may still finish with FASTCOD_OK).
 * FASTCOD_EINVAL if the id is unknown or already finished. */
int fastcod_server_cancel(fastcod_server *srv, uint64_t request_id);
int fastcod_server_get_stats(fastcod_server *srv, fastcod_server_stats *out);
/* Cancels every unfinished request, waits for the device work to drain and frees the server. */
int fastcod_server_destroy(fastcod_server *srv);

/*
 * Parcellation outputs of a connectivity matrix (Section 3, "Pie-glyphs": the single-colour map
 * shows each source voxel's most strongly connected region; a pie-glyph shows its relative
 * connectivity to every region).  For each row i of C:
 *   label_out[i]   = the lowest m with C[i][m] equal to the row maximum; -1 when no entry of the
 *                    row is positive
 *   frac_out[i][m] = C[i][m] / sum_m C[i][m], the quotient of the two integers taken in double and
 *                    rounded to float; 0 for a row whose sum is not positive
 *   sums_out[i]    = sum_m C[i][m] (int64)
 *   C [N][M] int32, label_out [N] int32, frac_out [N][M] float32, sums_out [N] int64: all device;
 *   any output may be NULL.  Asynchronous on `stream`.
 * Errors: EINVAL (N < 0, M < 1, N*M >= 2^31, C NULL with N > 0), EHIP.
 */
int fastcod_parcellate(const int32_t *C, int32_t N, int32_t M, int32_t *label_out, float *frac_out,
                       int64_t *sums_out, void *stream);

/*
 * Input check (synchronous): offsets[0] == 0 and nondecreasing, ROI values < N and label
 * values < M wherever they are >= 0.  Returns FASTCOD_OK or FASTCOD_ERANGE (detail in
 * fastcod_last_error).
 */
int fastcod_validate(const int64_t *offsets, int64_t n_streamlines, const int32_t *roi_index_vol,
                     const int32_t *target_label_vol, const int32_t dims[3], int32_t N, int32_t M,
                     void *stream);

/* Static description of a status code. */
const char *fastcod_strerror(int status);
/* Detail of the last failing call on this thread ("" if none). */
const char *fastcod_last_error(void);
/* Frees every cached workspace that no call is using (synchronises the devices that own them
 * first).  FASTCOD_EBUSY: a call on another thread was enqueueing with one of them at that moment;
 * that workspace was kept (the others are freed) -- call again once that call has returned.  The
 * fixed scratch area of fastcod_volume_count_noalloc is not a workspace and is never freed. */
int fastcod_release(void);

#ifdef __cplusplus
}
#endif

#endif /* FASTCOD_H */

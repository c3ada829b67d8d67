/*
 * discord.h -- C ABI of the MI355X (gfx950) discord-search library libdiscord.so.
 *
 * Problem (the paper's section 2.1): for a series T of m values and a window n,
 * the subsequences T_{i,n} = (t_i .. t_{i+n-1}), 0 <= i < N = m - n + 1, are
 * compared with the Euclidean distance of eq. (1); T_{j,n} is a non-self match
 * of T_{i,n} when |i - j| >= n.  The discord is the subsequence whose nearest
 * non-self match is farthest away.  The search follows PhiDD (Algorithm 2):
 * a preparation stage (z-normalisation statistics of eq. (2), PAA/SAX words of
 * eqs. (3)-(4), the word hash of eq. (9), Cand of eq. (7) and Index_Word of
 * eq. (10)) and a search stage (PotentialDiscord over Cand, Algorithm 3, then
 * RefineDiscord over the other rows, Algorithm 4) with early abandon against a
 * best-so-far.  Distances are compared squared and the root is taken once.
 *
 * Conventions
 *   - Indices are 0-based (the paper counts from 1).
 *   - Ties: the lowest index wins among maximal nearest-neighbour distances, and
 *     the lowest j among nearest neighbours.  Rows with no non-self match at all
 *     (possible only when 2n <= m <= 3n-2) take no part in the argmax.
 *   - z-normalisation is global (eq. (2)) by default; it is affine, so the argmax
 *     is taken on raw squared distances and `distance` = sqrt(d2) / sigma.  With
 *     opts.znorm = 1 every window is normalised on its own instead (see
 *     discord_opts), and `distance` = `distance_raw` = sqrt(d2).
 *   - The result is exact: every approximate (FP32 or split-BF16) decision is
 *     certified or redone in FP64 on the GPU before it is returned.
 *   - A negative status means no output was written.  No C++ exception crosses
 *     this boundary.  All functions are thread-safe for distinct plans; a plan
 *     must not be used from two threads at once.
 */
#ifndef DISCORD_H
#define DISCORD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* 2: discord_opts lost its unused `topk` field (the certification rescores
 * every row's witness in FP64 instead of the k best candidates of some rows). */
#define DISCORD_ABI_VERSION 4

/* ---- status codes ------------------------------------------------------- */
#define DISCORD_OK        0
#define DISCORD_EINVAL   -1  /* NULL series, n < 1, m < 2n, NaN/Inf in T, bad option */
#define DISCORD_ECONST   -2  /* sigma == 0: eq. (2) is undefined for a constant series */
#define DISCORD_ENOMEM   -3  /* device memory (or the caller's workspace) too small */
#define DISCORD_EDEVICE  -4  /* HIP runtime error; text in discord_plan_error() */
#define DISCORD_EBUSY    -5  /* server full or request not finished */
#define DISCORD_ERANGE   -6  /* size beyond a documented limit */

/* ---- options ------------------------------------------------------------- */
typedef enum {
    DISCORD_PREC_FP32   = 0,  /* FP32 direct form sum (a-b)^2 on the vector ALUs */
    DISCORD_PREC_BF16X3 = 1   /* centred split-BF16 hi/lo products on MFMA, FP32 accumulate */
} discord_precision;

/* Largest window the split-BF16 MFMA scan takes (ERANGE beyond it). */
#define DISCORD_MIXED_MAX_N 2048

typedef struct {
    int32_t precision;  /* discord_precision                                         */
    int32_t abandon;    /* 1: leave a row once a distance below the best-so-far appears
                           (Algorithms 1, 3, 4); 0: scan every pair (full scan)      */
    int32_t order;      /* visiting order; the result never depends on it:
                           1: PhiDD (Cand rows first, Algorithm 3; then each row's
                              same-word columns first, then matrix order, Alg. 4)
                           2: Cand rows first, then each row's columns nearest in
                              time first, alternating forward and backward
                           0: matrix order only                                    */
    int32_t paa_w;      /* PAA segments w of eq. (3) (1..8; min(w, n) is used)       */
    int32_t alphabet;   /* SAX alphabet size |A| of eq. (4) (2..8, |A|^w <= 256)      */
    int32_t probe_steps;/* abandon mode: the first window of every row's column
                           sequence, in steps of 512 columns; rows still live
                           then continue in later windows (0: library default,
                           2 (FP32) or 4 (split-BF16) for order 2, else 16)      */
    int32_t znorm;      /* which z-normalisation the distance uses:
                           0: the whole series once (eq. (2)); affine, so the
                              argmax is taken on raw squared distances
                           1: every window on its own (Algorithm 2's
                              Znormalize(S) read row by row): window i becomes
                              x_{i,k} = (t_{i+k} - mu_i) / sigma_i with mu_i,
                              sigma_i the eq. (2) statistics of that window
                              (two-pass, FP64); a flat window (sigma_i = 0)
                              becomes the zero vector.  Distances are between
                              normalised windows; d2 and distance are in those
                              units.  SAX words come from the same windows. */
} discord_opts;

/* Defaults: FP32, abandon on, order 2 (Cand first, then near-first columns),
 * w = |A| = 4 (section 3.1). */
void discord_default_opts(discord_opts* opts);

/* DISCORD_ABI_VERSION of the library actually loaded (a binding checks it
 * against the header it was written for). */
int32_t discord_abi_version(void);

/* ---- result -------------------------------------------------------------- */
typedef struct {
    int64_t  index;           /* discord row i (0-based)                            */
    int64_t  nn_index;        /* its nearest non-self match j (lowest j on ties)     */
    double   d2;              /* squared distance to it, FP64 (sequential sum): raw
                                 values, or normalised windows when opts.znorm = 1  */
    double   distance_raw;    /* sqrt(d2)                                           */
    double   distance;        /* sqrt(d2) / sigma: distance on the series of eq. (2);
                                 sqrt(d2) when opts.znorm = 1                       */
    double   mu, sigma;       /* eq. (2) statistics (FP64, two-pass)                 */
    double   max_rel_err;     /* largest relative error of an approximate NN value
                                 that was checked in FP64 during certification       */
    int32_t  certified;       /* 1: FP64 certificate complete (always, on success)   */
    int32_t  precision;       /* discord_precision used by the scan                  */
    uint64_t pairs_evaluated; /* pair distances computed by the approximate scan      */
    uint64_t rows_rescored;   /* rows whose exact NN was recomputed in FP64           */
    uint64_t rows_abandoned;  /* rows left early against the best-so-far              */
    uint64_t cand_rows;       /* |Cand| (eq. 7)                                       */
    double   ms_prepare;      /* device time of discord_prepare (HIP events)         */
    double   ms_search;       /* device time of discord_search (HIP events)          */
    double   ms_scan;         /* of which: the approximate scan launches, one event
                                 span from the first to the end of the last (the
                                 few-us window-decision kernels between them
                                 included)                                        */
    uint64_t scan_launches;   /* scan launches enqueued (the device-decided search
                                 enqueues a fixed number; those past the end of its
                                 loop find no work)                                 */
    int32_t  graph;           /* how the work was launched: 0 ordinary launches, 1
                                 captured into a HIP graph and launched, 2 a replay
                                 of a graph captured by an earlier call (see
                                 discord_search_graph and the serving loop)          */
    int32_t  reserved;        /* 0                                                   */
} discord_result;

typedef struct discord_plan_s* discord_plan;

/* Device bytes a plan for (m, n, opts) needs.  This is what discord_prepare
 * allocates (workspace == NULL) or requires of a caller workspace.  0 on
 * invalid arguments and on sizes discord_prepare refuses with ERANGE. */
size_t discord_workspace_bytes(int64_t m, int32_t n, const discord_opts* opts);

/* Preparation stage (Algorithm 2, first six steps).
 *   T          series of m float32 values, host or device pointer (detected with
 *              hipPointerGetAttributes); borrowed for the call and copied.
 *   opts       NULL for defaults.
 *   workspace  NULL: the plan allocates and owns its device memory.  Otherwise a
 *              device buffer of ws_bytes >= discord_workspace_bytes(), 256-byte
 *              aligned, owned by the caller and kept alive until release.
 *   stream     hipStream_t to run on, or NULL for a stream owned by the plan.
 *   out        receives the plan.
 * Errors: EINVAL, ECONST, ENOMEM, EDEVICE (see above). */
int discord_prepare(const float* T, int64_t m, int32_t n, const discord_opts* opts,
                    void* workspace, size_t ws_bytes, void* stream, discord_plan* out);

/* Search stage (Algorithms 3 and 4) and FP64 certification.  Blocks until the
 * result is on the host.  May be called repeatedly on one plan (each call redoes
 * the whole search; the prepared structures are reused).
 * Certification: the fully scanned row with the largest approximate NN is
 * rescanned in FP64 (exact NN L); every other row's witness distance is
 * recomputed in FP64 and clears the row when below L (or equal, at a higher
 * index); rows not cleared are rescanned in FP64; the answer is the FP64 argmax
 * with the lowest index on ties.  No error bound of the approximate arithmetic
 * is relied on. */
int discord_search(discord_plan plan, discord_result* out);

/* The same search, run from a HIP graph: the first call on a plan captures the
 * whole search (every launch, the device-side decisions between them and the
 * readback of the answer; nothing in it waits for the host) and later calls
 * replay it, so a resident plan searched again costs one graph launch and one
 * synchronisation.  Same result as discord_search, bit for bit.  The graph
 * and a small pinned readback block belong to the plan (freed by
 * discord_release).  ms_scan is 0 (no per-launch events inside the graph);
 * ms_search brackets the graph launch.  Errors: those of discord_search, and
 * EDEVICE if capture or instantiation fails (the plan stays usable with
 * discord_search). */
int discord_search_graph(discord_plan plan, discord_result* out);

/* One call from a series to its certified discord: the computation and result
 * of discord_prepare + discord_search with `opts`, enqueued as one sequence on
 * the device with one host synchronisation (the statistics of eq. (2) are
 * checked from the same readback as the answer), and no plan left behind.
 * The PhiDD order (opts.order = 1) synchronises once more, after the
 * preparation (its sequences need the bucket sizes on the host).
 *   T          m float32 values, host or device pointer.
 *   opts       NULL for defaults.
 *   workspace  a device buffer of ws_bytes >= discord_workspace_bytes(m, n,
 *              opts), 256-byte aligned, owned by the caller and free for the
 *              duration of the call; NULL: the call allocates and frees one.
 *   stream     hipStream_t to run on (NULL: the null stream); synchronised
 *              before the call returns.
 *   out        receives the result.  ms_scan spans the scan launches (HIP
 *              events); ms_search spans preparation and search and ms_prepare
 *              is 0, except in the PhiDD order, whose two stages are timed
 *              apart as in discord_prepare and discord_search.
 * Errors: those of discord_prepare and discord_search (ENOMEM also for a
 * workspace that is too small or misaligned); the text is in
 * discord_plan_error(NULL). */
int discord_search_once(const float* T, int64_t m, int32_t n, const discord_opts* opts,
                        void* workspace, size_t ws_bytes, void* stream, discord_result* out);

/* Frees the plan and the device memory it owns.  NULL is ignored. */
void discord_release(discord_plan plan);

/* Static text for a status code. */
const char* discord_strerror(int status);

/* Detail of the last error on this plan ("" if none).  With plan == NULL: the
 * detail of the calling thread's last failed discord_prepare,
 * discord_search_once or discord_search_series_noalloc. */
const char* discord_plan_error(discord_plan plan);

/* The inner breakpoints beta_1..beta_{alpha-1} of eq. (4) (N(0,1) quantiles
 * k/alpha) that the library's SAX step uses; out holds alpha-1 doubles.
 * alpha in 2..8. */
int discord_sax_breakpoints(int32_t alpha, double* out);

/* One-shot: prepare + search with default options on a library stream. */
int discord_search_series(const float* T, int64_t m, int32_t n, int64_t* index,
                          double* distance);

/* For callers that cannot allocate (code under stream capture, tight serving
 * loops, hosts that forbid allocation): prepare + search of one series, the
 * same computation and result as discord_prepare + discord_search with `opts`,
 * with no device allocation, no stream or event creation and no heap plan.
 * The plan lives in a static device array of DISCORD_NOALLOC_MAX_BYTES that
 * each GPU the library runs on holds until the process ends; its address is
 * taken once per device on the first call there.
 *   T       m float32 values, host or device pointer (a host series goes
 *           through the runtime's own copy).
 *   opts    NULL for defaults.
 *   stream  hipStream_t to run on (NULL: the null stream); synchronised before
 *           the call returns.
 *   out     receives the result; ms_prepare / ms_search / ms_scan are 0 (no
 *           events are taken).
 * Errors: those of discord_prepare / discord_search, and ERANGE when the plan
 * (discord_workspace_bytes(m, n, opts)) is larger than the array; the text is
 * in discord_plan_error(NULL).  Calls on one GPU share its array: calls that
 * overlap on the same GPU race (serialise them). */
#define DISCORD_NOALLOC_MAX_BYTES ((size_t)32 << 20)
int discord_search_series_noalloc(const float* T, int64_t m, int32_t n,
                                  const discord_opts* opts, void* stream,
                                  discord_result* out);

/* ---- introspection of the prepared and searched state (for verification) -- */
typedef enum {
    DISCORD_FIELD_WORDS       = 0,  /* int32[N]    word id of each row, eqs. (3)(4)(9)   */
    DISCORD_FIELD_HIST        = 1,  /* int32[|A|^w] word frequencies, eq. (8)           */
    DISCORD_FIELD_CAND        = 2,  /* int32[cand] Cand, ascending, eq. (7)             */
    DISCORD_FIELD_CSR_OFFSETS = 3,  /* int32[|A|^w + 1] Index_Word offsets, eq. (10)    */
    DISCORD_FIELD_CSR_MEMBERS = 4,  /* int32[N]    Index_Word members (ascending/word)  */
    DISCORD_FIELD_NN_APPROX   = 5,  /* float[N]    approximate NN d^2 of the last search
                                       (full rows) or the abandon distance             */
    DISCORD_FIELD_NN_WITNESS  = 6,  /* int32[N]    j attaining NN_APPROX (-1: none)     */
    DISCORD_FIELD_ROW_STATE   = 7,  /* int32[N]    0 not scanned, 1 full scan, 2 abandoned */
    DISCORD_FIELD_ROW_MEAN    = 8,  /* double[N]   mean of each row (FP64)              */
    DISCORD_FIELD_ROW_CNORM   = 9,  /* double[N]   centred squared norm of each row     */
    DISCORD_FIELD_ROW_SIGMA   = 10, /* double[N]   standard deviation of each row, FP64,
                                       sqrt(ROW_CNORM / n) (opts.znorm = 1 plans only;
                                       EINVAL otherwise)                                */
    DISCORD_FIELD_ROW_BOUND   = 11  /* float[N]    a lower bound of each row's NN d^2: n
                                       times the squared gap from its mean to the means
                                       of its non-self rows, at bin resolution; the
                                       search completes the rows with the largest bound
                                       first (opts.znorm = 0 plans only; EINVAL
                                       otherwise)                                       */
} discord_field;

/* Number of elements of a field (Cand length after prepare; N or table sizes
 * otherwise); negative status on error. */
int64_t discord_plan_count(discord_plan plan, int32_t field);

/* Copies a field to host memory; `bytes` must be >= count * element size. */
int discord_plan_copy(discord_plan plan, int32_t field, void* host_dst, size_t bytes);

/* Exact FP64 nearest non-self match of the listed rows (the rescoring kernel of
 * the certification, exposed for verification): d2_out[r], j_out[r] (-1: none).
 * rows / outputs are host pointers of `count` elements. */
int discord_rows_nn_fp64(discord_plan plan, const int64_t* rows, int64_t count,
                         double* d2_out, int64_t* j_out);

/* ---- compute-unit-limited streams (scalability study) ----------------------
 * The paper reports speedup and parallel efficiency against the number of
 * cores it runs on (section 4, its scalability experiments).  On the GPU the
 * unit is the compute unit (CU): a search on a stream from
 * discord_stream_create_cu_limited runs every kernel on `cus` CUs of the
 * current device only, so timing the same search at several CU counts gives
 * that study.
 *
 * discord_cu_mask (host only, no device call) writes the CU mask used:
 * `cus` bits spread evenly over the device's `xccs` accelerator dies, so
 * that every die keeps cus / xccs CUs whether the runtime assigns mask bit b
 * to die b / (total_cus / xccs) (contiguous) or to die b % xccs
 * (interleaved).  Mask bit b is bit b % 32 of words[b / 32].
 * Requires xccs >= 1, total_cus a multiple of xccs with (total_cus / xccs) a
 * multiple of xccs, cus a multiple of xccs with 1 <= cus <= total_cus, and
 * nwords >= ceil(total_cus / 32).  Returns the number of words written, or
 * EINVAL.
 *
 * discord_stream_create_cu_limited creates such a stream (default priority,
 * non-blocking) on the current device, reads its mask back and checks that it
 * holds exactly `cus` CUs.  Returns OK, EINVAL (sizes as above, with the
 * device's CU and die counts), or EDEVICE (the runtime refused the mask or
 * changed it; no stream is left behind).  The caller owns the stream and
 * releases it with discord_stream_destroy (which synchronises it first). */
int discord_cu_mask(int32_t total_cus, int32_t xccs, int32_t cus, uint32_t* words,
                    int32_t nwords);
int discord_stream_create_cu_limited(int32_t cus, void** stream_out);
int discord_stream_destroy(void* stream);

/* ---- serving ---------------------------------------------------------------
 * The paper has no serving layer; this is a request loop around the same
 * prepare + search path.  Requests (T, m, n) of uneven size are queued in
 * arrival order and admitted, strictly first-in first-out, as soon as a slot is
 * free and their device footprint (discord_workspace_bytes, rounded up to 256 B)
 * fits in the free part of one device arena of `hbm_budget_bytes` allocated at
 * creation.  Each slot is a host worker thread with its own HIP stream (default
 * priority), so the kernels of all admitted requests run concurrently on the
 * device; a request's prepared structures stay resident in its arena block from
 * prepare to the end of its search, and the block returns to the arena when the
 * request completes.  A request's result depends only on its own series: the
 * requests share no device state besides the arena, whose blocks are disjoint.
 * A failing request completes with its status and never disturbs the others.
 * A slot that serves requests of one shape keeps its arena block (a request
 * whose footprint equals the slot's previous one gets that block back when it
 * is free) and replays its preparation and search as one captured HIP graph:
 * the second request of a shape on a slot is captured, later ones are replays
 * (result.graph = 1, 2; 0 for ordinary launches, and always for order = 1).
 * All server functions are thread-safe. */
typedef struct discord_server_s* discord_server;

typedef struct {
    size_t       hbm_budget_bytes; /* size of the device arena                         */
    int32_t      slots;            /* requests in flight at once, 1..64                */
    int32_t      max_queued;       /* waiting requests beyond which submit returns
                                      EBUSY (0: 65536)                                */
    discord_opts opts;             /* options of every request                         */
} discord_server_config;

/* One request as an executor sees it. */
typedef struct {
    uint64_t     tag;        /* caller's tag from discord_server_submit               */
    const float* T;          /* host copy of the series (m values), valid for the call */
    int64_t      m;
    int32_t      n;
    int32_t      slot;       /* worker slot running the request, 0..slots-1           */
    void*        workspace;  /* device block of ws_bytes inside the arena (NULL when the
                                server was created with an executor: virtual arena) */
    size_t       ws_offset;  /* offset of the block in the arena                       */
    size_t       ws_bytes;   /* the request's footprint                                */
} discord_request;

/* An executor runs one admitted request on the calling worker thread and fills
 * `out`; it returns a status and may write a message of at most `detail_len`
 * bytes (NUL-terminated) to `detail`. */
typedef int (*discord_executor_fn)(void* ctx, const discord_request* req,
                                   const discord_opts* opts, discord_result* out,
                                   char* detail, size_t detail_len);

typedef struct {
    uint64_t tag;
    int32_t  status;        /* DISCORD_OK or the request's error                      */
    int32_t  slot;
    size_t   ws_offset;     /* arena block the request held                           */
    size_t   ws_bytes;
    double   t_submit_ms;   /* server clock (steady, ms since creation)               */
    double   t_admit_ms;    /* slot and arena block granted                            */
    double   t_done_ms;     /* result on the host                                      */
    discord_result result;  /* valid when status == DISCORD_OK                         */
    char     detail[96];    /* error text ("" on success)                              */
} discord_completion;

typedef struct {
    uint64_t submitted;     /* accepted by submit                                      */
    uint64_t rejected;      /* refused by submit (EINVAL, ENOMEM, EBUSY)               */
    uint64_t completed;     /* completions produced, successful or not                 */
    uint64_t failed;        /* completions with a negative status                      */
    int32_t  queued;        /* waiting for admission now                               */
    int32_t  running;       /* admitted and not yet complete now                       */
    int32_t  peak_running;
    int32_t  slots;
    size_t   budget_bytes;
    size_t   bytes_in_use;
    size_t   peak_bytes_in_use;
    double   busy_ms;       /* sum over completed requests of (done - admit): divided
                               by elapsed_ms it is the mean admitted concurrency      */
    double   elapsed_ms;    /* server clock now                                        */
} discord_server_stats;

/* Server on the current device: allocates the arena (ENOMEM if it cannot) and
 * starts cfg->slots workers, each running prepare + search of its requests on
 * its own stream with a pinned host staging buffer. */
int discord_server_create(const discord_server_config* cfg, discord_server* out);

/* The same scheduler with a caller-supplied executor instead of the GPU path
 * (for cost models and host tests): no device memory is allocated and blocks
 * are offsets in a virtual arena of hbm_budget_bytes. */
int discord_server_create_with_executor(const discord_server_config* cfg,
                                        discord_executor_fn exec, void* ctx,
                                        discord_server* out);

/* Queues a request; T is a host pointer of m float32 values, copied before the
 * call returns.  Returns DISCORD_OK, EINVAL (NULL T, n < 1, m < 2n, m beyond
 * the length limit), ERANGE (split-BF16 with n > DISCORD_MIXED_MAX_N), ENOMEM
 * (footprint larger than the whole arena: it could never run, or no host memory
 * for the copy) or EBUSY (queue full).  Errors found later (NaN/Inf in T, a
 * constant series, a device error) arrive as the request's completion status. */
int discord_server_submit(discord_server s, const float* T, int64_t m, int32_t n,
                          uint64_t tag);

/* Moves up to `max` completions, oldest first, into `out`; waits up to
 * timeout_ms (0: no wait, at most 60000) for the first one.  *count receives the
 * number written. */
int discord_server_poll(discord_server s, discord_completion* out, int32_t max,
                        int32_t timeout_ms, int32_t* count);

int discord_server_get_stats(discord_server s, discord_server_stats* out);

/* Stops admitting, waits for the running requests, drops the queued ones and
 * frees everything.  NULL is ignored. */
void discord_server_destroy(discord_server s);

#ifdef __cplusplus
}
#endif
#endif /* DISCORD_H */

/*
 * lpf.h -- C ABI of the MI355X (gfx950) hot path for real-time detection of
 * dispersed radio transients in image cubes (Ruhe et al., "Detecting
 * Dispersed Radio Transients in Real Time Using Convolutional Neural
 * Networks", arXiv:2103.15418).
 *
 * Per 1 s time step a stream delivers one image cube X_t of B subbands x H x W
 * pixels (Sec. 2.1: the pipeline's input at time t is a B x D x D cube).  The
 * library runs the paper's per-step stages on the GPU:
 *   lpf_ingest_frame  quality control (App. A) and the image cache (Sec. 2.2)
 *   lpf_detect        centre/spread estimates, sigma threshold, peak map
 *                     (Sec. 2.1.1-2.1.2), duplicate removal, association and
 *                     monitoring (Sec. 2.2)
 *   lpf_extract_flux  box-maximum flux per band, backward fill, dynamic
 *                     spectra (Sec. 2.2, Fig. 3)
 *   lpf_infer         the CNN giving mean and Cholesky factor of the physical
 *                     parameters (Sec. 2.3.3)
 *
 * Conventions
 *  - Every call returns an int status (LPF_OK = 0 or a negative LPF_E*) and
 *    never throws; lpf_last_error() gives the context's last message.
 *  - Memory: everything passed in stays owned by the caller.  Device memory
 *    the library uses lives in caller-allocated workspaces (sizes from
 *    lpf_workspace_size / lpf_model_workspace_size); the workspace must stay
 *    allocated and untouched until the context / model is destroyed.  The
 *    context and model structs themselves are library-owned host memory.
 *  - Streams: each context is bound to one hipStream_t at creation; all its
 *    device work is ordered on that stream.  Only calls that return host data
 *    synchronise with it (noted per call).
 *  - Pixel layout: float32, band-major, row-major: cube[(b*H + i)*W + j].
 *  - Time steps t must strictly increase; a gap marks the skipped steps
 *    missing in the dynamic spectra.
 *  - Non-finite input is not an error: quality control discards the band.
 *  - Call order per step: ingest -> detect -> extract_flux; infer after
 *    extract_flux.  Violations return LPF_ESTATE.
 *  - A context is not thread-safe; distinct contexts may be used from
 *    distinct threads.
 *  - After a HIP error a context is poisoned: every later call returns
 *    LPF_EDEVICE.
 */
#ifndef LPF_H
#define LPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lpf_ctx lpf_ctx;     /* one per image stream (opaque)        */
typedef struct lpf_model lpf_model; /* CNN weights, shareable across ctxs  */

enum {
    LPF_OK = 0,
    LPF_EINVAL = -1,  /* bad argument or configuration                       */
    LPF_ENOMEM = -2,  /* workspace too small                                 */
    LPF_EFULL = -3,   /* source or peak capacity reached; the step completed,
                         excess dropped and counted (see lpf_status)          */
    LPF_EORDER = -4,  /* t not increasing                                     */
    LPF_EDEVICE = -5, /* HIP error; the context is poisoned                   */
    LPF_ESTATE = -6   /* call order violated                                  */
};
/* Background kernel (Sec. 2.1.1): Gaussian, square uniform, or circular
 * uniform (disk of radius bg_halfwidth: offsets with u^2 + v^2 <= k^2; float32
 * filters with one clip iteration, k <= 32). */
enum { LPF_KERNEL_GAUSS = 0, LPF_KERNEL_BOX = 1, LPF_KERNEL_DISK = 2 };
enum { LPF_PREC_FP32 = 0, LPF_PREC_BF16 = 1, LPF_PREC_FP16 = 2 };

/* Method parameters.  Names follow Sec. 2.1-2.2 and App. A. */
typedef struct {
    int32_t B, H, W;          /* subbands (1..16), image rows, columns (1..4096) */
    const uint8_t* sky_mask;  /* host [H][W] 0/1, copied at create; NULL = all  */
    const int32_t* grid_rows; /* host [B] rows of the 16-row network input that
                                 the bands occupy; NULL = b * (16 / B)          */
    float kappa;              /* threshold in spreads: y = x > c + kappa sqrt(s) */
    float bg_sigma;           /* Gaussian width s, pixels                       */
    int32_t bg_halfwidth;     /* kernel half-width k; <= 0 -> ceil(3 s); <= 40  */
    int32_t kernel;           /* LPF_KERNEL_GAUSS, _BOX (square) or _DISK         */
    int32_t clip_iters;       /* sigma-clip iterations, 1..16                    */
    int32_t peak_halfwidth;   /* max-filter half-width (paper: 3), 1..8          */
    int32_t flux_halfwidth;   /* flux box half-width, 0..8                       */
    float dup_radius;         /* cross-band duplicate radius, pixels            */
    float assoc_radius;       /* association radius, pixels                     */
    int32_t monitor_steps;    /* measured while t - t_last_det <= this          */
    int32_t backfill_steps;   /* backward fill depth (image cache holds +1)     */
    int32_t ring_len;         /* dynamic-spectrum window; must be 64            */
    float qc_band_z;          /* band-mean robust z threshold (App. A: 5)       */
    float qc_rms_z;           /* band-RMS robust z threshold; <= 0 disables     */
    float qc_rms_floor;       /* RMS scale floor as a fraction of the median    */
    float qc_pixel_zeta;      /* per-pixel running z threshold                  */
    int32_t qc_warmup;        /* accepted frames before the pixel test arms     */
    int32_t max_sources;      /* source table capacity, 1..65536                */
    int32_t peak_cap;         /* per band per step; B * peak_cap <= 8192        */
    int32_t filter_precision; /* LPF_PREC_FP32, or BF16 / FP16 operands on MFMA  */
    int32_t debug_planes;     /* 1: also keep S (and the clip mask) readable    */
    int32_t pipeline_ingest;  /* 1: ingest and QC of the next step run on a
                                 stream of the context's own, beside this
                                 step's catalogue and flux (see
                                 lpf_ingest_frame); the image cache holds one
                                 step more.  0: everything on the context's
                                 stream                                        */
    /* detection variants (Sec. 2.1.1 and Sec. 2.2 readings) */
    float psf_sigma;          /* > 0: detection runs on the image correlated
                                 with a Gaussian PSF of this width (pixels) over
                                 the sky mask and normalised like C (a matched
                                 filter for point sources); flux still reads
                                 the quality-controlled image.  0: off        */
    int32_t psf_halfwidth;    /* PSF kernel half-width; <= 0 -> ceil(4 psf_sigma); <= 40 */
    int32_t flux_bg_width;    /* > 0: flux = box maximum minus the mean of the
                                 annulus of this width around the box (local
                                 background); 0: raw box maximum              */
} lpf_config;

/* One peak of the map P = Q and Y (Sec. 2.1.2) with the local estimates. */
typedef struct {
    int32_t band, row, col;
    float x;   /* pixel value                       */
    float c;   /* centre estimate C at the pixel    */
    float s;   /* spread estimate S at the pixel    */
    float sig; /* (x - c) / sqrt(s); +inf if s = 0  */
} lpf_peak;

enum { LPF_EVENT_NEW = 1, LPF_EVENT_ENDED = 2 };
/* A source-table event of this step (Sec. 2.2). */
typedef struct {
    int32_t id, row, col, event;
    int64_t t_first, t_last_det, t_end; /* t_end: last measured step (ended) */
} lpf_source;

/* Per-step counters, filled by lpf_status (synchronises). */
typedef struct {
    int64_t t;
    uint32_t rejected_bands;  /* QC decision of the last ingested step          */
    uint32_t overflow_bands;  /* bands whose peak count exceeded peak_cap:
                                 their peaks are dropped whole                 */
    int32_t n_peaks, n_kept, n_new, n_ended, n_measured, n_dropped, n_live;
} lpf_status_t;

/* Fills cfg with the defaults: kappa 4.5, s 8, k ceil(3s), Gaussian, 1
 * iteration, k_peak 3, k_flux 2, radii 3, monitor 31, backfill 32, ring 64,
 * QC 5 / 5 / 0.05 / 30 / 8, max_sources 8192, peak_cap 512.  Host only. */
int lpf_config_default(lpf_config* cfg, int32_t B, int32_t H, int32_t W);

/* Bytes of device workspace a context with cfg needs.  Host only; no device
 * call.  LPF_EINVAL for an invalid configuration. */
int lpf_workspace_size(const lpf_config* cfg, size_t* bytes);

/* Creates a context.  dev_workspace: device memory of at least
 * lpf_workspace_size bytes, 256-byte aligned, caller-owned, outliving the
 * context.  hip_stream: a hipStream_t (NULL = default stream).  Copies the
 * sky mask and initialises state on the stream (asynchronously). */
int lpf_create(const lpf_config* cfg, void* dev_workspace, size_t bytes, void* hip_stream,
               lpf_ctx** out);
void lpf_destroy(lpf_ctx* ctx);

/* Quality control (App. A) of the cube for step t and its entry into the
 * image cache.  cube: [B][H][W] float32, device memory if cube_on_device,
 * else host memory (copied before return).  A device cube is only read.
 * Ordering: after earlier work on the context's stream; with
 * pipeline_ingest = 1 only after the previous step's filters instead (the
 * first ingest after create waits for the whole stream), so a device cube
 * must then be complete before the previous lpf_detect call was made, or be
 * produced on a stream the caller has synchronised.
 * Per band: mean and RMS over all pixels (float64 sums), robust z of each
 * across bands, max |zeta| of sky pixels against the running mean/std of
 * accepted steps; a band failing any test (or holding a non-finite value)
 * is discarded (treated as all zeros downstream) and kept out of the
 * running statistics.  rejected_out (nullable): the band bitmask; when
 * non-null the call synchronises.  LPF_EORDER if t does not increase. */
int lpf_ingest_frame(lpf_ctx* ctx, int64_t t, const float* cube, int32_t cube_on_device,
                     uint32_t* rejected_out);

/* Source detection (Sec. 2.1) on the last ingested step, then duplicate
 * removal, association and monitoring (Sec. 2.2).  Asynchronous unless an
 * output is requested.  peaks_out (nullable, host, cap entries): all peaks
 * of the step in (band, row, col) order, *n_peaks their total count.
 * events_out (nullable, host, ev_cap entries): sources opened at this step
 * (in id order) then episodes ended at this step (in id order); *n_events.
 * Returns LPF_EFULL (after completing the step) if a band overflowed
 * peak_cap or the source table was full. */
int lpf_detect(lpf_ctx* ctx, lpf_peak* peaks_out, int32_t cap, int32_t* n_peaks,
               lpf_source* events_out, int32_t ev_cap, int32_t* n_events);

/* Flux (Sec. 2.2): the maximum of the quality-controlled image within the
 * (2k+1)^2 box (clipped to the image) around each measured source, every
 * band, into the source's dynamic-spectrum ring; new sources are also
 * measured on the cached steps [max(t - backfill, first t), t - 1].
 * Device-only and asynchronous. */
int lpf_extract_flux(lpf_ctx* ctx);

/* Batch forms of the three per-step calls for n contexts (several image
 * streams of uneven B, H, W; Sec. 3.5: every stream must keep up with its
 * cadence) as grouped launches: each stage runs as one kernel launch over up
 * to 8 contexts, whose workgroups find their context's arguments in a table
 * passed with the launch (the filter passes group contexts with the same
 * float32 strip kernel, one clip iteration and equal taps; others run their
 * own launches).  Results are bitwise those of the per-context calls.
 * Requirements: the contexts are distinct, were created on one hipStream_t
 * (the launches go there) and have pipeline_ingest = 0 (LPF_EINVAL
 * otherwise).  Every context is checked before anything is launched: a call
 * order or time order violation of any context returns LPF_ESTATE /
 * LPF_EORDER with nothing done.  Nothing is read back: per-context counters
 * and outputs come from lpf_status, lpf_read_spectrum and lpf_infer*.
 * lpf_ingest_batch: t[n] steps, cubes[n] cubes (device memory if
 * cubes_on_device, else host memory copied before return, which then
 * synchronises). */
int lpf_ingest_batch(lpf_ctx* const* ctxs, const int64_t* t, const float* const* cubes,
                     int32_t cubes_on_device, int32_t n);
int lpf_detect_batch(lpf_ctx* const* ctxs, int32_t n);
int lpf_extract_flux_batch(lpf_ctx* const* ctxs, int32_t n);

/* Counters of the last step; synchronises. */
int lpf_status(lpf_ctx* ctx, lpf_status_t* out);

/* Dynamic spectrum of a held source: the ring_len steps ending at its last
 * measured step.  out: host [B][ring_len] float32 (invalid cells 0);
 * valid: host [B][ring_len] 0/1 (nullable); t_last (nullable): that step.
 * Synchronises.  LPF_EINVAL if the id is not held. */
int lpf_read_spectrum(lpf_ctx* ctx, int32_t source_id, float* out, uint8_t* valid,
                      int64_t* t_last);

/* ---- parameter inference (Sec. 2.3.3) ------------------------------------ */

/* Weights blob: little-endian float32 in this order (PyTorch layouts):
 * conv1.w[32][1][3][3] conv1.b[32] conv2.w[32][32][3][3] conv2.b[32]
 * conv3.w[64][32][3][3] conv3.b[64] conv4.w[64][64][3][3] conv4.b[64]
 * fc1.w[128][65536] fc1.b[128] fc2.w[14][128] fc2.b[14], followed by one
 * float: the leaky-rectifier slope alpha (0 = plain rectifier).  Flatten
 * order before fc1 is (channel, row, column) of the 64 x 16 x 64 map. */
size_t lpf_model_weights_bytes(void);

/* Device workspace for a model of the given precision serving batches of up
 * to max_batch windows (larger synchronous requests are processed in chunks).
 * The model also allocates, once at creation, its inference stream, events
 * and four pinned host result blocks of 16 max_batch + 4 words each. */
int lpf_model_workspace_size(int32_t precision, int32_t max_batch, size_t* bytes);

/* Uploads and re-lays-out the weights (host blob) into dev_workspace on
 * hip_stream and synchronises.  precision: LPF_PREC_FP32 / BF16 / FP16 for
 * the convolutions and dense layers (accumulation is always float32). */
int lpf_model_create(const void* weights, size_t bytes, int32_t precision, int32_t max_batch,
                     void* dev_workspace, size_t ws_bytes, void* hip_stream, lpf_model** out);
void lpf_model_destroy(lpf_model* model);

/* Runs the network (Sec. 2.3.2-2.3.3) on the dynamic spectra (Sec. 2.2,
 * Fig. 3) of sources of one or more contexts, batched together on the
 * model's own inference stream (ordered after each context's stream by
 * events).  source_ids: NULL = every episode that ended at the context's
 * last detect (all contexts); else n_ids ids of ctxs[0] (n_ctx must be 1).
 * Outputs (host): mu_out [N][4] (DM, width, amplitude, arrival), L_out
 * [N][10] packed row-major lower triangle with softplus diagonal, src_out
 * [N][2] (context index, source id), rows in (context, id) order for
 * source_ids == NULL; at most cap rows.  *n_out: rows written.  Synchronises
 * (once, on the results, when the ended episodes fit the model's batch). */
int lpf_infer(lpf_ctx* const* ctxs, int32_t n_ctx, const lpf_model* model,
              const int32_t* source_ids, int32_t n_ids, float* mu_out, float* L_out,
              int32_t* src_out, int32_t cap, int32_t* n_out);

/* The network alone on device windows: windows [n][16][64] float32, mu_out
 * [n][4], L_out [n][10] device float32.  Asynchronous with respect to the
 * host; ordered after earlier work on hip_stream, and later work on
 * hip_stream is ordered after it. */
int lpf_infer_windows(const lpf_model* model, const float* windows, int32_t n, float* mu_out,
                      float* L_out, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the network
 * on n <= LPF_STATIC_MAX_WINDOWS device windows, as lpf_infer_windows
 * computes it, with its intermediate buffers (activations and fc1 partials)
 * in a file-scope device array of the library (about 18 MiB,
 * one copy per GPU, held until the process ends) instead of the model's
 * workspace.  Launches directly on hip_stream; allocates nothing and makes
 * no allocating call.  The model still supplies the weights; windows, mu_out
 * and L_out are caller-owned device buffers as in lpf_infer_windows.
 * LPF_EINVAL for n > LPF_STATIC_MAX_WINDOWS or null buffers, LPF_EDEVICE on
 * a HIP error.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (different streams or threads) race and must be
 * serialised by the caller. */
enum { LPF_STATIC_MAX_WINDOWS = 32 };
int lpf_infer_windows_static(const lpf_model* model, const float* windows, int32_t n, float* mu_out,
                             float* L_out, void* hip_stream);

/* Asynchronous form of lpf_infer over the episodes that ended at the last
 * detect of each context (Sec. 2.2 episode end -> Sec. 2.3 inference): the
 * counts stay on the device, the windows are gathered there (into buffers of
 * the ticket: on the context's own stream when n_ctx is 1, else on the
 * model's stream), the network runs on the model's stream and the results
 * are copied into a pinned host slot; nothing waits.  For one context with
 * pipeline_ingest = 1 the network is launched after the centre pass of that
 * context's next lpf_detect (beside its spread pass and catalogue), or by
 * the context's next lpf_infer_async, lpf_infer_collect of the ticket or
 * lpf_destroy of the context if one of those comes first.  Each context's later
 * work is ordered after the gather, so the caller may ingest the next frame
 * at once.  *ticket
 * identifies the results for lpf_infer_collect.  At most 4 tickets may be
 * outstanding per model (LPF_EFULL otherwise).  Episodes beyond the model's
 * max_batch are not inferred; lpf_infer_collect reports them. */
int lpf_infer_async(lpf_ctx* const* ctxs, int32_t n_ctx, lpf_model* model, int64_t* ticket);

/* Waits for a ticket of lpf_infer_async and writes its rows as lpf_infer
 * does (host outputs, (context, id) order, at most cap rows, *n_out rows).
 * Returns LPF_EFULL when more episodes ended than the model's max_batch
 * (the first max_batch in gather order were inferred), LPF_EINVAL for an
 * unknown or already collected ticket.  Tickets may be collected in any
 * order. */
int lpf_infer_collect(lpf_model* model, int64_t ticket, float* mu_out, float* L_out, int32_t* src_out,
                      int32_t cap, int32_t* n_out);

/* ---- candidates, alerts and state persistence ---------------------------- */

/* Candidate selection on the network's outputs (Sec. 2.3.1: nearby noise is
 * not dispersed, so low dispersion measures are excluded; Sec. 3.3-3.4: on
 * real data the inferred DM is kept above 50 and candidates are ranked by the
 * inferred standard deviation of the DM, large values marking false
 * positives).  mu [n][4] and L [n][10] as lpf_infer returns them (host).
 * sigma_DM = sqrt(Sigma_00) with Sigma = L L^T, i.e. |L_00|.  Keeps the rows
 * with mu_DM > dm_min and sigma_DM <= sigma_max, ordered by sigma_DM
 * ascending (ties: row); idx_out [n] receives their row indices, *n_out
 * their count; sigma_out [n] (nullable) every row's sigma_DM.  Host only. */
int lpf_select_candidates(const float* mu, const float* L, int32_t n, float dm_min, float sigma_max,
                          int32_t* idx_out, float* sigma_out, int32_t* n_out);

/* Image data of a candidate for an alert (Sec. 1: a trigger saves the data of
 * interest): the (2 half + 1)^2 box around (row, col) of the cached
 * quality-controlled cube of each step t_first .. t_first + n_steps - 1.
 * out: host [n_steps][B][2 half + 1][2 half + 1] float32, zero outside the
 * image, in rejected bands and for steps no longer cached; have (nullable):
 * host [n_steps], 1 where the step was cached.  half <= 32, n_steps <= the
 * cache depth (backfill_steps + 1, + 1 with pipeline_ingest).  Synchronises. */
int lpf_read_cutouts(lpf_ctx* ctx, int32_t row, int32_t col, int32_t half, int64_t t_first, int32_t n_steps,
                     float* out, uint8_t* have);

/* Checkpoint of a context's state between steps (after lpf_extract_flux, or
 * before the first ingest): image cache, running QC statistics, source table,
 * dynamic-spectrum rings, the last step's lists and counters, and the step
 * bookkeeping, as one host byte block of lpf_checkpoint_size bytes.
 * lpf_checkpoint_save synchronises (LPF_ESTATE inside a step, LPF_ENOMEM for
 * a short buffer).  lpf_checkpoint_load restores it into a context created
 * with the same configuration and sky mask that has taken no step yet
 * (LPF_EINVAL for another configuration or mask, LPF_ESTATE after a step);
 * the stream then continues with bitwise the results the saved context
 * would give.  Inference tickets are not part of a context's state. */
int lpf_checkpoint_size(lpf_ctx* ctx, size_t* bytes);
int lpf_checkpoint_save(lpf_ctx* ctx, void* host_buf, size_t bytes);
int lpf_checkpoint_load(lpf_ctx* ctx, const void* host_buf, size_t bytes);

/* ---- inspection (tests, diagnostics) ------------------------------------- */
enum {
    LPF_DBG_BANDSTATS = 1, /* double [B][6]: mean, rms, z_mean, z_rms, zeta_max, nonfinite */
    LPF_DBG_WELFORD_MEAN = 2, /* float [B][H][W] running mean (accepted steps)   */
    LPF_DBG_WELFORD_M2 = 3,   /* float [B][H][W] running M2                      */
    LPF_DBG_WELFORD_N = 4,    /* int32 [B] accepted-step counts                   */
    LPF_DBG_CENTRE = 5,       /* float [B][H][W] C of the last iteration          */
    LPF_DBG_SPREAD = 6,       /* float [B][H][W] S (needs debug_planes)           */
    LPF_DBG_CLIPMASK = 7,     /* uint8 [B][H][W] Y (needs debug_planes or iters>1) */
    LPF_DBG_CACHE = 8,        /* float [B][H][W] cached cube of the last step     */
    LPF_DBG_PEAKS = 9,        /* lpf_peak [n_peaks] of the last detect, (band, row,
                                 col) order (n_peaks from lpf_status)             */
    LPF_DBG_EVENTS = 10,      /* lpf_source [n_new + n_ended] of the last detect:
                                 new sources in id order, then ended episodes in
                                 the device's list order                          */
    LPF_DBG_PREFILTERED = 11  /* float [B][H][W] PSF-correlated detection image
                                 of the last detect (psf_sigma > 0)               */
};
/* Copies an internal buffer to host memory (bytes must match); synchronises.
 * Rows of rejected bands in the centre/spread planes are unspecified. */
int lpf_debug_read(lpf_ctx* ctx, int32_t what, void* host_out, size_t bytes);

/* Stage timing with HIP events recorded around each selected stage's kernels
 * on the stream they run on (diagnostics: every event pair costs the stream a
 * few microseconds, so time only the stages of interest in a timed run).
 * Stages: 0 ingest pass, 1 QC decision, 2 centre filter, 3 spread filter +
 * threshold + peaks (and further clip iterations), 4 association,
 * 5 flux + backfill, 6 network (recorded on the model's stream for ctxs[0]).
 * stages: bit i selects stage i (LPF_PROFILE_ALL for every stage, 0 = off). */
enum { LPF_STAGE_COUNT = 7, LPF_PROFILE_ALL = (1 << 7) - 1 };
int lpf_profile_enable(lpf_ctx* ctx, int32_t stages);
/* Sums the recorded stage times (ms) and counts since the last read and
 * clears them; synchronises.  ms / counts: host arrays of LPF_STAGE_COUNT. */
int lpf_profile_read(lpf_ctx* ctx, double* ms, int64_t* counts);

int lpf_sync(lpf_ctx* ctx);
const char* lpf_last_error(const lpf_ctx* ctx);

/* ---- serving loop -----------------------------------------------------------
 * Several image streams of different shapes served concurrently on one GPU
 * (Sec. 3.5: the pipeline must keep up with the 1 s cadence of the stream).
 * A dispatcher thread owned by the server works in rounds: each round takes
 * the next frame of every idle stream that has one and runs ingest, detect
 * and extract_flux for all of them as batch calls (lpf_*_batch: grouped
 * launches on the server's one HIP stream), then one pooled network ticket
 * over the episodes that ended in those streams (lpf_infer_async).  Up to
 * four rounds are in flight; a frame is done when its round's network
 * results are on the host.  A stream's next frame joins a round after its
 * previous frame is done.  Streams are active while the sum of their
 * workspaces fits the HBM budget; a stream that does not fit is refused or
 * waits in admission order until closed streams free their share. */
typedef struct lpf_server lpf_server;

typedef struct {
    int32_t stream_id;
    int64_t t;
    int64_t arrival_ns, done_ns; /* host steady clock, as given / measured     */
    uint32_t rejected_bands;
    int32_t n_peaks, n_new, n_ended;
    int32_t status;              /* LPF_OK or the error of this frame's round:
                                    LPF_EFULL if more episodes ended in the
                                    round than the model's max_batch (those
                                    beyond it are not inferred)              */
} lpf_frame_result;

/* model: network for the pooled inference (not owned; the server uses its
 * asynchronous tickets, so the model must serve no other caller meanwhile).
 * record != 0 keeps every frame's peaks, events and inference outputs for
 * lpf_server_fetch (tests; adds synchronisation per round).  The server
 * creates one HIP stream (default priority) and its dispatcher thread. */
int lpf_server_create(const lpf_model* model, size_t hbm_budget_bytes, int32_t record, lpf_server** out);
void lpf_server_destroy(lpf_server* srv);
/* Admits a stream with configuration cfg (pipeline_ingest is ignored: served
 * contexts run on the server's stream).  dev_workspace: caller-owned device
 * memory of at least lpf_workspace_size(cfg) bytes (256-byte aligned) that
 * outlives the stream, or NULL to let the server allocate it when the stream
 * becomes active and free it at close.  The workspace size counts against
 * the budget while the stream is active.  If it does not fit (or other
 * streams are already waiting): with queue = 0 LPF_ENOMEM and nothing is
 * kept; with queue = 1 the stream waits (frames may be submitted and are
 * held) until lpf_server_close of other streams frees enough budget.
 * *stream_id: handle for submit / close; *active (nullable): 1 if active
 * now, 0 if waiting.  The sky mask and grid rows are copied. */
int lpf_server_admit(lpf_server* srv, const lpf_config* cfg, void* dev_workspace, size_t ws_bytes,
                     int32_t queue, int32_t* stream_id, int32_t* active);
/* Waits for the stream's submitted frames (a waiting stream's frames are
 * dropped), destroys it, releases its budget share (and its workspace if the
 * server allocated it) and activates waiting streams that now fit. */
int lpf_server_close(lpf_server* srv, int32_t stream_id);
/* Queues one frame.  cube: [B][H][W] float32 (device memory if on_device);
 * it must stay valid until the frame is reported done.  arrival_ns: the
 * frame's arrival time on the host steady clock (latency origin).  t must
 * increase per stream (a frame out of order fails its round). */
int lpf_server_submit(lpf_server* srv, int32_t stream_id, int64_t t, const float* cube, int32_t on_device,
                      int64_t arrival_ns);
/* Completed frames since the last poll (at most cap); non-blocking. */
int lpf_server_poll(lpf_server* srv, lpf_frame_result* out, int32_t cap, int32_t* n);
/* Blocks until every submitted frame of the active streams is done;
 * LPF_ESTATE if waiting streams still hold frames. */
int lpf_server_drain(lpf_server* srv);
/* Recorded outputs of frame (stream_id, t) (record mode): peaks in (band,
 * row, col) order, events as lpf_detect, inference rows (mu [4], L [10], id)
 * for the episodes that ended at t.  Any output pointer may be NULL. */
int lpf_server_fetch(lpf_server* srv, int32_t stream_id, int64_t t, lpf_peak* peaks, int32_t peak_cap,
                     int32_t* n_peaks, lpf_source* events, int32_t ev_cap, int32_t* n_events, float* mu,
                     float* L, int32_t* ids, int32_t inf_cap, int32_t* n_inf);
/* Budget in use (workspaces of active streams), the budget, active streams. */
int lpf_server_usage(const lpf_server* srv, size_t* used, size_t* budget, int32_t* n_streams);
/* Host time server steady clock (ns), for arrival stamps. */
int64_t lpf_now_ns(void);

#ifdef __cplusplus
}
#endif
#endif /* LPF_H */

/*
 * wdd.h - C ABI of the live Wigner Distribution Deconvolution per-frame update
 * on AMD Instinct MI355X (gfx950).
 *
 * The method (Bangun et al., "Wigner Distribution Deconvolution Adaptation for
 * Live Ptychography Reconstruction", arXiv 2212.01309):
 *   - each detector frame I_s is projected onto a reduced Hermite-Gauss basis,
 *     h_s = Phi^T vec(I_s)                          (Section 5, operator H);
 *   - it is weighted by its scan-position phase and summed into the spectrum
 *     A[v, k] += F[v, s] h_s[k],  F = F_y (x) F_x   (Section 6.1, eq. outer_prod;
 *     modified-WDD algorithm, outer-product step);
 *   - on demand the spectrum is Wiener-deconvolved by the probe's reduced
 *     Wigner function, D[v] = sum_k W[v, k] A[v, k] (pre-computed Wiener filter
 *     algorithm; modified-WDD algorithm, deconvolution and summation steps);
 *   - and inverse transformed, O~ = conj(IDFT2(D)) / sqrt(|D[0]|)
 *     (eq. extract; final step of the modified-WDD algorithm).
 *
 * Conventions (fixed readings of points the paper leaves open):
 *   - detector frames are row-major [ny][nx]; the aperture sits at the probe's centre
 *     (ny/2, nx/2 for fftshifted frames of a centred beam);
 *   - scan positions are 0-based integer raster indices (y, x) on an sy x sx grid
 *     with step `step_px` object pixels; repeated positions are summed;
 *   - scan frequencies are 0-based DFT indices; the scan DFT is unitary;
 *   - the K basis functions are psi_{n_y}(y) psi_{n_x}(x), n_y, n_x < L =
 *     ceil(sqrt(K)), ordered by (max(n_y, n_x), n_y + n_x, n_y); psi_n are
 *     L2-normalised Hermite functions at t = (i - c) / sigma, c the aperture centre,
 *     each sampled column normalised on the grid; sigma defaults to R / sqrt(2L - 1);
 *   - eps = eps_rel * max_{v,k} |Phi^T vec(Y_v)|^2;
 *   - only frequencies whose shifted aperture overlaps the unshifted one on a
 *     detector pixel are kept (Section 6.2); D is zero elsewhere.
 *
 * Memory: complex values are interleaved float pairs (re, im).  "Device"
 * pointers are HIP device allocations on the plan's device; "host" pointers are
 * ordinary host memory.  The caller owns every buffer it passes; the plan owns
 * its device state.  All calls return a wdd_status; on failure
 * wdd_last_error() returns a message for the calling thread.  A plan is used
 * by one host thread at a time; distinct plans are independent.
 */
#ifndef WDD_H
#define WDD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A push call returns once its work is queued.  At most this many pushes of a plan are
 * queued and not yet run: a push waits, if need be, until the one this many pushes
 * earlier has been read. */
#define WDD_MAX_PUSHES_IN_FLIGHT 64

typedef enum {
  WDD_OK = 0,
  WDD_EINVAL = -1,   /* bad argument, size or option */
  WDD_ENOMEM = -2,   /* host or device allocation failed */
  WDD_ERANGE = -3,   /* a scan position outside the raster; nothing was applied */
  WDD_EDEVICE = -4,  /* a HIP call failed; the plan is now unusable */
  WDD_EBUSY = -5,    /* reserved */
  WDD_ESTATE = -6    /* call not valid in the plan's state (e.g. after a device error) */
} wdd_status;

typedef enum { WDD_U16 = 0, WDD_F32 = 1 } wdd_dtype;

/* Arithmetic of the projection's first (N^2 L) stage.  WDD_FP32: FP32 MFMA.  The others
 * need uint16 frames and use BF16 or FP16 MFMA with FP32 accumulation: counts are split
 * exactly into two digits, the basis is rounded to one (BF16, FP16) or two (_HILO:
 * hi + lo) 16-bit parts.  Everything after the projection stays FP32. */
typedef enum { WDD_FP32 = 0, WDD_BF16_HILO = 1, WDD_FP16_HILO = 2, WDD_BF16 = 3, WDD_FP16 = 4 } wdd_precision;

/* Fourier-space probe: amplitude * 1[|u| <= radius] * exp(-i defocus_edge_rad |u|^2 / radius^2),
 * u = detector pixel - (center_y, center_x).  Initial probe of the pre-computed Wiener
 * filter algorithm (initialisation step 1), generated from the aperture radius; its centre
 * is where the unscattered beam meets the detector, (ny/2, nx/2) for fftshifted frames of a
 * centred beam.  The Hermite-Gauss basis is centred there too (Section 5: the functions sit
 * at the centre of the bright-field disc).  The kept-frequency test is exact when the centre
 * is a multiple of 1/2 pixel and the detector shifts are dyadic (power-of-two sizes);
 * otherwise pixels exactly on a rim are decided in FP64 rounding. */
typedef struct {
  double radius_px;
  double center_y, center_x;
  double defocus_edge_rad;
  double amplitude;
} wdd_probe;

/* Equispaced raster of sy x sx positions, `step_px` object pixels apart (Section 2). */
typedef struct {
  int32_t sy, sx;
  double step_px;
} wdd_scan;

/* Detector of ny x nx pixels; frames arrive as `dtype` (uint16 counts or float32). */
typedef struct {
  int32_t ny, nx;
  int32_t dtype; /* wdd_dtype */
} wdd_detector;

/* Where the Wiener filter is applied.  WDD_ORDER_SPECTRUM: frames are accumulated into the
 * spectrum A[v, k] (resident in HBM, a sufficient statistic) and the filter is applied at each
 * snapshot.  WDD_ORDER_OBJECT: the filter is applied per frame and the object spectrum D[v] is
 * accumulated directly, as written in the modified-WDD algorithm (Section 6.3); A is not kept,
 * so wdd_get_accumulator and wdd_update_probe are unavailable.  Both give the same result. */
typedef enum { WDD_ORDER_SPECTRUM = 0, WDD_ORDER_OBJECT = 1 } wdd_order;

/* The reduced basis Phi (Sections 4-5).  WDD_BASIS_HERMITE_GAUSS: K real Hermite-Gauss
 * functions (1 <= K <= 256, shell order).  WDD_BASIS_FOURIER: the full Fourier basis
 * Phi[q, k] = exp(+2 pi i (q_y k_y / ny + q_x k_x / nx)) / (ny nx), k = k_y nx + k_x, with
 * K = ny nx: the method then computes conventional WDD exactly (Section 5 remarks that the
 * Fourier basis is the conventional case).  Needs ny, nx powers of two in [8, 64], FP32
 * precision; projections h are complex. */
typedef enum { WDD_BASIS_HERMITE_GAUSS = 0, WDD_BASIS_FOURIER = 1 } wdd_basis;

typedef struct {
  double eps_rel;     /* Wiener regularisation relative to the largest |Y^B|^2; default 0.01 */
  double sigma_px;    /* basis width in detector pixels; <= 0 selects radius / sqrt(2L - 1) */
  int32_t precision;  /* wdd_precision; default WDD_FP32 */
  int32_t max_batch;  /* largest n accepted by wdd_push; default 256 */
  int32_t order;      /* wdd_order; default WDD_ORDER_SPECTRUM */
  int32_t basis;      /* wdd_basis; default WDD_BASIS_HERMITE_GAUSS */
  int32_t pipeline;   /* 0 (default), 1 or 2: pipelined pushes, see below */
} wdd_options;

/* Pipelined pushes (wdd_options.pipeline = 1).  The update of a batch (its accumulation into
 * D, Section 6.3, modified-WDD algorithm, the loop body) is held back and runs in the next
 * push's launch, beside that push's projection: the two are independent, and the
 * projection's frame stream from HBM then overlaps the update's first phase.  Every call
 * that waits for the plan's stream or reads or changes its state (wdd_snapshot, wdd_sync,
 * wdd_spectrum, wdd_get_*, wdd_profile_read, checkpoints, wdd_reset, wdd_destroy) first runs
 * a held update, so results are those of unpipelined pushes up to FP32 rounding (the
 * projection sums its tiles in another order; a snapshot taken while a batch is held gets
 * the display's first pass from that batch's update, as wdd_push_snapshot does, so push +
 * snapshot then gives wdd_push_snapshot's image).  A WDD_OUT_DEVICE_DEFERRED snapshot after
 * push i is written during push i + 2 (its update runs in push i + 1's launch, its display's
 * last pass in push i + 2's), or by such a call.  pipeline = 2 adds a stage: the x-DFT of a
 * batch's projections along the scan rows (Section 6.1, the F_x factor of eq. outer_prod),
 * formed once per kept v_x, runs one launch ahead of the update, which then streams W at
 * once; a push's launch holds the update of batch i - 2, the x-DFT of batch i - 1 and the
 * projection of batch i, and a deferred image lands three pushes later.  With no x-DFT to
 * repeat, the update is cut into longer chunks (at least four rounds of its frequency loop), so
 * D is the same as with pipeline = 1 while the images, whose first display pass is summed over
 * one partial row per chunk, differ from it by FP32 rounding.  Batches on more than 16 scan
 * rows run unpipelined after the held ones.  Needs WDD_ORDER_OBJECT, the Hermite-Gauss
 * basis, uint16 frames of 32..256 columns in multiples of 32 and at most 256 rows (128 with a
 * reduced-precision projection), and power-of-two scan sides with Sy <= 1024; other plans:
 * WDD_EINVAL. */

typedef struct {
  int64_t n_freq;        /* number of kept scan frequencies */
  int32_t k;             /* reduced basis size */
  int32_t l;             /* 1D basis functions per axis */
  double sigma_px;       /* basis width actually used */
  double eps_abs;        /* absolute Wiener regularisation */
  uint64_t frames_seen;  /* frames pushed since the plan was made or reset */
  int64_t device_bytes;  /* device memory held by the plan */
  int32_t update_chunks; /* object order: workgroups of a row pass (runs of kept frequencies of one v_x) */
  int32_t display_slots; /* object order: partial display rows kept per v_x (0: the two-pass display) */
  int32_t pipelined;     /* pipeline stages of pushes (wdd_options.pipeline) */
  int32_t kept_columns;  /* object order: the kept v_x (two-stage pipelining forms one x-DFT per column
                            per batch; the update's chunks take update_chunks / kept_columns each) */
} wdd_plan_info;

typedef struct wdd_tables_s* wdd_tables_t;
typedef struct wdd_plan_s* wdd_plan_t;

/* Message describing the last failure on the calling thread ("" if none).  The
 * string stays valid until the thread's next wdd_* call. */
const char* wdd_last_error(void);

/* Fills *opts with the defaults listed in wdd_options. */
wdd_status wdd_default_options(wdd_options* opts);

/* ------------------------------------------------------------------------- */
/* Host tables (FP64; no device needed).  The pre-computed quantities of the
 * pre-computed Wiener filter algorithm: the kept frequencies (Section 6.2), the
 * sampled Hermite functions (Section 5) and W_v = conj(Y^B_v) / (|Y^B_v|^2 + eps)
 * with Y^B_v = Phi^T vec(Y_v), Y_v(q) = P(q) conj(P(q + q_v)).                  */

/* Builds the tables.  K in [1, 256]; sy, sx in [1, 4096]; ny, nx in [1, 1024]
 * with nx a multiple of 8; the aperture must cover at least one detector pixel.  `opts`
 * may be NULL (defaults).  WDD_EINVAL on bad arguments, WDD_ENOMEM if the tables do not
 * fit in host memory. */
wdd_status wdd_tables_build(const wdd_probe* probe, const wdd_scan* scan, const wdd_detector* det,
                            int32_t K, const wdd_options* opts, wdd_tables_t* out);

/* n_freq, k, l, sigma_px and eps_abs of the tables (other fields zero). */
wdd_status wdd_tables_info(wdd_tables_t t, wdd_plan_info* info);

/* Copies the tables to host arrays; any pointer may be NULL to skip it.
 *   freqs  int32  [n_freq][2]   (v_y, v_x), sorted by v_y then v_x; (0, 0) first
 *   psi_y  double [ny][l]       sampled, grid-normalised Hermite functions
 *   psi_x  double [nx][l]
 *   pairs  int32  [k][2]        (n_y, n_x) of each basis function
 *   w      double [n_freq][k][2] Wiener filter (re, im)
 * With the Fourier basis l = 0 and psi_y, psi_x, pairs are left untouched.      */
wdd_status wdd_tables_export(wdd_tables_t t, int32_t* freqs, double* psi_y, double* psi_x,
                             int32_t* pairs, double* w);

wdd_status wdd_tables_free(wdd_tables_t t);

/* ------------------------------------------------------------------------- */
/* Live reconstruction on the current HIP device.                            */

/* Creates a plan for one acquisition: the pre-computed Wiener filter algorithm (its
 * initialisation from the aperture, the kept frequencies of Section 6.2, the reduced
 * probe Wigner functions and W) built in FP64 on the host, uploaded to the device as FP32,
 * and a zeroed accumulator.  The plan keeps its FP64 tables (wdd_plan_export).
 *   probe, scan, det  acquisition settings (host structs, read during the call);
 *   K                 reduced basis size (1..256, or ny nx with the Fourier basis);
 *   opts              NULL for the defaults of wdd_default_options;
 *   hip_stream        the hipStream_t all of the plan's work is ordered on; NULL makes the
 *                     plan create its own (non-blocking) stream.
 * WDD_EINVAL (bad settings), WDD_ENOMEM (host or device memory), WDD_EDEVICE. */
wdd_status wdd_plan(const wdd_probe* probe, const wdd_scan* scan, const wdd_detector* det, int32_t K,
                    const wdd_options* opts, void* hip_stream, wdd_plan_t* out);

/* Adds n frames (Section 6.3, modified-WDD algorithm, the body of its loop over frames):
 * projection onto the reduced basis (Section 5, operator H), weighting by the scan
 * position's column of the unitary scan DFT (Section 6.1, eq. outer_prod) and accumulation
 * into the spectrum A (or, in WDD_ORDER_OBJECT, the Wiener-filtered object spectrum D).
 *   frames  n x ny x nx values of the detector dtype; device memory if
 *           frames_on_device != 0 (must stay valid until the work completes:
 *           wdd_sync, a blocking snapshot, or WDD_MAX_PUSHES_IN_FLIGHT further
 *           pushes), else host memory (copied before the call returns).
 *   pos_yx  host int32 [n][2] scan indices.
 * Batches whose frames lie on at most 16 scan rows are accumulated through the
 * Kronecker factorisation F = F_y (x) F_x (per-row x-DFT, then one pass over the
 * spectrum); others through the direct phase-weighted sum.  Both give the same
 * result up to rounding.
 * Asynchronous on the plan stream.  n = 0 is a no-op.  WDD_EINVAL if n < 0 or
 * n > max_batch; WDD_ERANGE if any position is outside the raster, in which case
 * no frame of the call is applied. */
wdd_status wdd_push(wdd_plan_t p, const void* frames, const int32_t* pos_yx, int32_t n,
                    int32_t frames_on_device);

/* wdd_push followed by wdd_snapshot (Section 6.3, modified-WDD algorithm: the loop body
 * and the final summation, inverse transform and conjugation), with the same arguments and
 * results.  When the
 * batch uses the row-factored update (it touches at most 16 scan rows), the Wiener
 * reduction is done in the same pass over the spectrum.  In object order with power-of-two
 * scan sides (Sy <= 1024) the update also performs the first pass of the display's inverse
 * DFT, split over its workgroups; the image then equals that of wdd_push + wdd_snapshot up
 * to FP32 rounding (a different summation order), and a wdd_snapshot before the next push
 * returns it again bit for bit. */
wdd_status wdd_push_snapshot(wdd_plan_t p, const void* frames, const int32_t* pos_yx, int32_t n,
                             int32_t frames_on_device, float* out, int32_t out_on_device, uint64_t* frames_seen);

/* Where a snapshot is written (the out_on_device argument).
 *   WDD_OUT_HOST          host memory; the call blocks until `out` is written.
 *   WDD_OUT_DEVICE        device memory (8-byte aligned); blocks until it is written.
 *   WDD_OUT_DEVICE_ASYNC  device memory (8-byte aligned); returns once the work is
 *                         enqueued on the plan's stream.  `out` (which must stay valid)
 *                         is complete after wdd_sync, or once the plan's stream passes
 *                         this point; frames_seen then counts the frames enqueued.
 *   WDD_OUT_DEVICE_DEFERRED  as WDD_OUT_DEVICE_ASYNC, except that the image (of this
 *                         point's spectrum) may be written by the plan's next push, in
 *                         one of that push's launches (its projection; for detectors of
 *                         more than 128 rows in object order, its first update: one
 *                         kernel boundary fewer per pipelined step; with pipelined
 *                         pushes, by the push after next, or the third with two
 *                         stages), or else by the next
 *                         call that waits for the plan's stream or changes its state
 *                         (wdd_snapshot, wdd_sync, wdd_get_*, wdd_profile_read,
 *                         checkpoints, wdd_update_probe, wdd_reset, wdd_destroy).  `out`
 *                         is complete after wdd_sync.  Where the display's last pass
 *                         cannot wait (the Fourier basis, scans whose Sx is not a power
 *                         of two, detectors of more than 128 rows in spectrum order) it
 *                         is queued at once, as WDD_OUT_DEVICE_ASYNC. */
typedef enum { WDD_OUT_HOST = 0, WDD_OUT_DEVICE = 1, WDD_OUT_DEVICE_ASYNC = 2, WDD_OUT_DEVICE_DEFERRED = 3 } wdd_out_kind;

/* Takes a snapshot of all frames pushed so far (Section 6.3, modified-WDD algorithm, the
 * steps after the loop; eq. extract): Wiener reduction D[v] = sum_k W[v,k] A[v,k], inverse
 * unitary DFT over the scan, conjugation and normalisation by sqrt(|D[0]|).  Reflects
 * exactly the frames pushed before the call.  Writes sy x sx complex values
 * (interleaved float, row-major [y][x]) to `out`, a wdd_out_kind place given by
 * out_on_device (any other value: WDD_EINVAL).
 * Object pixel mapping: out[y][x] is the object at scan position (y, x) shifted
 * by the probe's centre (ny/2, nx/2) within its window.  frames_seen may be NULL. */
wdd_status wdd_snapshot(wdd_plan_t p, float* out, int32_t out_on_device, uint64_t* frames_seen);

/* The plan's pinned host buffer of sy x sx complex values that host snapshots are
 * written through.  Passing it as `out` (out_on_device = 0) skips the final host
 * copy.  Owned by the plan, valid until wdd_destroy; each host snapshot
 * overwrites it. */
wdd_status wdd_snapshot_buffer(wdd_plan_t p, float** host_out);

/* Test hook (blocking): the Wiener-reduced spectrum D on the kept frequencies (eq. extract
 * before the inverse transform; Section 6.3, modified-WDD algorithm, summation step),
 * n_freq complex values in the order of wdd_plan_export's freqs, as computed by the last
 * snapshot (in WDD_ORDER_OBJECT D is always current).  d_out: device memory if
 * on_device != 0, else host memory. */
wdd_status wdd_spectrum(wdd_plan_t p, float* d_out, int32_t on_device);

/* Test hook: the FP64 tables the plan was built from and uploaded (pre-computed Wiener
 * filter algorithm; Sections 5 and 6.2).  Any pointer may be NULL to skip it.
 *   phi    double [ny nx][K] the reduced basis, Phi[y nx + x][k] = psi_{n_y(k)}[y] psi_{n_x(k)}[x]
 *          (Hermite-Gauss), or [ny nx][K][2] (re, im) with the Fourier basis;
 *   w      double [n_freq][K][2] the Wiener filter W;
 *   freqs  int32  [n_freq][2] the kept frequencies (v_y, v_x), 0-based DFT indices sorted by
 *          v_y then v_x, (0, 0) first: the rows of W, D and A.
 * The device holds W rounded to FP32 (wdd_get_wiener) and the sampled psi rounded to FP32. */
wdd_status wdd_plan_export(wdd_plan_t p, double* phi, double* w, int32_t* freqs);

/* Inspection (blocking): the Wiener filter as the device holds it, n_freq x K complex
 * float values (FP32 rounding of wdd_plan_export's w). */
wdd_status wdd_get_wiener(wdd_plan_t p, float* w_out, int32_t on_device);

/* Inspection (blocking): the accumulated spectrum A, n_freq x k complex values
 * (WDD_ESTATE in WDD_ORDER_OBJECT). */
wdd_status wdd_get_accumulator(wdd_plan_t p, float* a_out, int32_t on_device);

/* Inspection (blocking): the projections h of the last pushed batch, n x k floats
 * (n = size of that batch). */
wdd_status wdd_get_projection(wdd_plan_t p, float* h_out, int32_t on_device);

wdd_status wdd_plan_get_info(wdd_plan_t p, wdd_plan_info* info);

/* Per-stage device time, measured with HIP events recorded on the plan stream
 * around each kernel launch while profiling is enabled. */
typedef struct {
  double project_ms;     /* frame decode + basis projection */
  double accumulate_ms;  /* update of D (object order; the scan x-DFT fused in) or of A (spectrum
                            order: direct, or row-factored after the rowdft stage, with the Wiener
                            reduction when fused) */
  double wiener_ms;      /* Wiener reduction (when not fused) */
  double display_ms;     /* inverse DFT, conjugation and normalisation */
  int64_t project_launches, accumulate_launches, wiener_launches, display_launches;
  int64_t factored_launches; /* accumulate launches that took the row-factored form */
  double rowdft_ms;          /* per-row scan x-DFT of the spectrum-order row-factored update */
  int64_t rowdft_launches;
} wdd_profile;

/* Stages selectable for timing (bit mask). */
enum {
  WDD_STAGE_PROJECT = 1,
  WDD_STAGE_ACCUMULATE = 2,
  WDD_STAGE_WIENER = 4,
  WDD_STAGE_DISPLAY = 8,
  WDD_STAGE_ROWDFT = 16,
  WDD_STAGE_ALL = 31
};

/* Times the stages in the mask `stages` (0 turns timing off) and zeroes the totals.
 * Each timed launch adds two event records to the plan stream. */
wdd_status wdd_profile_enable(wdd_plan_t p, int32_t stages);

/* Times only one push in every `period` (>= 1; default 1), with the snapshot that follows
 * it, so that the event records disturb a long run less.  Zeroes the totals.  Counts in
 * wdd_profile are then of the sampled launches. */
wdd_status wdd_profile_period(wdd_plan_t p, int32_t period);

/* Totals since profiling was enabled (blocks until the timed work has finished). */
wdd_status wdd_profile_read(wdd_plan_t p, wdd_profile* out);

/* Re-deconvolution: replaces the Wiener filter by the one of `probe` (same aperture
 * radius and centre; defocus and amplitude may change) and `eps_rel`, built in FP64 as at plan
 * creation.  The accumulated spectrum A is kept (it does not depend on the probe), so
 * the next snapshot deconvolves every frame seen so far with the new filter without
 * re-reading them (Section 10: probe update; Algorithm "pre-computed Wiener filter").
 * WDD_EINVAL if the radius differs; WDD_ESTATE in WDD_ORDER_OBJECT. */
wdd_status wdd_update_probe(wdd_plan_t p, const wdd_probe* probe, double eps_rel);

/* Checkpoint of the live state (the spectrum A, or D in WDD_ORDER_OBJECT, and the frame
 * count: a sufficient statistic of all frames pushed).  wdd_checkpoint_size gives the byte size of the
 * image; wdd_checkpoint_save writes it to host memory (blocking); wdd_checkpoint_load
 * restores it into a plan of the same geometry and basis (WDD_EINVAL otherwise). */
wdd_status wdd_checkpoint_size(wdd_plan_t p, size_t* bytes);
wdd_status wdd_checkpoint_save(wdd_plan_t p, void* host_buf, size_t bytes);
wdd_status wdd_checkpoint_load(wdd_plan_t p, const void* host_buf, size_t bytes);

/* Zeroes the spectrum and the frame count (asynchronous): a new acquisition on the same
 * plan (Section 6.3, modified-WDD algorithm, the accumulator's initialisation). */
wdd_status wdd_reset(wdd_plan_t p);

/* Waits for all work queued on the plan stream; device frames and asynchronous outputs of
 * earlier calls may be reused afterwards. */
wdd_status wdd_sync(wdd_plan_t p);

/* Releases the plan (waits for its work first) and all its device and host memory.  NULL
 * is accepted. */
wdd_status wdd_destroy(wdd_plan_t p);

/* The display of a spectrum given on the whole scan grid (eq. extract; the final step of
 * the modified-WDD algorithm, Section 6.3): out = conj(IDFT2_unitary(D)) / sqrt(|D[0, 0]|),
 * all zeros when D[0, 0] = 0.
 *   spectrum  device, sy x sx complex values (interleaved float, row-major [v_y][v_x], 0-based
 *             DFT indices; zero outside the kept frequencies), 8-byte aligned; read only;
 *   out       device, sy x sx complex values [y][x], 8-byte aligned; may not overlap spectrum;
 *   hip_stream  the hipStream_t the work is queued on (NULL: the null stream).
 * 1 <= sy, sx <= 4096.  Asynchronous: returns once the work is queued; out is complete when
 * the stream reaches this point.  The scratch (two sy x sx grids and the twiddles) is taken
 * with hipMallocAsync and returned with hipFreeAsync on the same stream.  Stateless: calls on
 * different streams are independent.  WDD_EINVAL (sizes, null or misaligned pointers),
 * WDD_ENOMEM, WDD_EDEVICE. */
wdd_status wdd_display(const float* spectrum, int32_t sy, int32_t sx, float* out, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): wdd_display with the same arguments and
 * result, whose scratch is a fixed array in device memory that each GPU the library runs
 * on holds until the process ends (16.8 MB), so the call allocates nothing.  sy sx <=
 * 1 048 576 (e.g. 1024 x 1024) and sides <= 4096, else WDD_EINVAL.  All calls on one GPU
 * share that array: calls that overlap in time on one GPU (different streams, or host
 * threads) race and must be ordered by the caller; calls queued on one stream are ordered
 * by it.  Nothing in the array needs to start at zero. */
wdd_status wdd_display_noalloc(const float* spectrum, int32_t sy, int32_t sx, float* out, void* hip_stream);

/* Device memory for plans created after this call (tables, spectrum, grids, device
 * staging; not pinned host buffers) comes from alloc(bytes, ctx) and goes back through
 * release(ptr, ctx) when the plan is destroyed, after its stream has drained: a caller
 * with its own pool (a framework's caching allocator) lends it to the library.
 * alloc must return memory of the current device aligned to 256 bytes, or NULL; NULL
 * makes the plan's creation fail with WDD_ENOMEM, unaligned memory is released again and
 * WDD_EINVAL returned.  alloc = NULL restores hipMalloc / hipFree.  Process-wide and
 * thread-safe; a plan keeps the allocator it was created with.  WDD_EINVAL if alloc is
 * given without release. */
typedef void* (*wdd_alloc_fn)(size_t bytes, void* ctx);
typedef void (*wdd_release_fn)(void* ptr, void* ctx);
wdd_status wdd_set_allocator(wdd_alloc_fn alloc, wdd_release_fn release, void* ctx);

/* ------------------------------------------------------------------------- */
/* Field-of-view patches (Section 10, Discussion: a large field of view subdivided into
 * patches that are reconstructed independently and then merged, so that the cost grows
 * with the number of patches instead of with the square of the raster).  Reading of the
 * paper: patches are Py x Px sub-rasters whose origins step by (Py - overlap_y,
 * Px - overlap_x) from 0, the last one on each axis placed at S - P; every patch is a live
 * WDD of its own raster (object order), a frame entering every patch that contains its
 * position, at the local position; the merged image is the weighted mean of the patch images
 * with separable trapezoid windows min(1, (i + 1) / (o + 1), (P - i) / (o + 1)), which
 * de-weight each patch's edges (where its own scan DFT wraps around) wherever another patch
 * covers them.  A single patch covering the raster is the plain plan's result. */
typedef struct {
  int32_t py, px;                /* patch size in scan positions, 1 <= p <= the raster's side */
  int32_t overlap_y, overlap_x;  /* positions neighbouring patches share, 0 <= overlap < p */
} wdd_patch_geometry;

typedef struct wdd_patches_s* wdd_patches_t;

/* Creates a patch set for the whole raster `scan` (arguments as wdd_plan; the Hermite-Gauss
 * basis, object order, pushes not pipelined; all patches share one set of tables built for
 * the patch raster).
 * WDD_EINVAL for a geometry that does not fit the raster. */
wdd_status wdd_patches_create(const wdd_probe* probe, const wdd_scan* scan, const wdd_detector* det, int32_t K,
                              const wdd_patch_geometry* geo, const wdd_options* opts, void* hip_stream,
                              wdd_patches_t* out);

/* Adds n device frames (contiguous, 16-byte aligned; valid until the stream passes this
 * point) at host positions pos_yx [n][2] of the whole raster: each frame is projected once
 * and enters every patch that contains it.  Asynchronous.  WDD_ERANGE (nothing applied) for
 * a position off the raster; WDD_EINVAL for n outside [0, max_batch]. */
wdd_status wdd_patches_push(wdd_patches_t s, const void* frames, const int32_t* pos_yx, int32_t n);

/* The merged image of all frames pushed so far, sy x sx complex (interleaved float) on the
 * whole raster, into host memory (WDD_OUT_HOST, blocking) or device memory (WDD_OUT_DEVICE,
 * blocking; WDD_OUT_DEVICE_ASYNC, queued).  Pixel (y, x) is the object at scan position
 * (y, x) shifted by the probe centre, as for a plan. */
wdd_status wdd_patches_snapshot(wdd_patches_t s, float* out, int32_t out_on_device, uint64_t* frames_seen);

/* Patch grid, kept frequencies per patch and device memory held (any pointer may be NULL). */
wdd_status wdd_patches_info(wdd_patches_t s, int32_t* npatch_y, int32_t* npatch_x, int64_t* n_freq,
                            int64_t* device_bytes);

/* Waits for all work queued by the patch set. */
wdd_status wdd_patches_sync(wdd_patches_t s);

/* Releases the patch set (waits for its work first).  NULL is accepted. */
wdd_status wdd_patches_destroy(wdd_patches_t s);

/* ------------------------------------------------------------------------- */
/* Serving: many concurrent acquisitions on one GPU (the live update of Section 6.3 run
 * for several acquisitions at once; each keeps its own spectrum, Section 6.1).
 *
 * Each acquisition is a plan (spectrum resident in HBM).  wdd_server_open admits an
 * acquisition if the device memory of all open plans stays within the budget and
 * returns WDD_EBUSY otherwise (the caller retries after another closes); the plan itself
 * (FP64 tables, allocations, upload of W) is then made on a worker thread, and frames
 * submitted meanwhile wait in the queue.  Frames are submitted as device memory and
 * queued; wdd_server_step takes every queued frame of every ready acquisition (continuous
 * batching) and snapshots the acquisitions whose last snapshot is older than the snapshot
 * interval.  With WDD_SERVE_GROUPED (the default) Hermite-Gauss acquisitions are pushed
 * together in rounds: one projection launch for up to one batch of each (per frame type
 * and arithmetic), then per row pass one update launch over all object-order spectra and
 * one row-DFT and one A-update launch over all spectrum-order ones (the Wiener reduction
 * fused into the last pass before a snapshot); WDD_SERVE_GRAPH captures a round as a HIP
 * graph and replays it with updated arguments.  Fourier-basis acquisitions, and all of
 * them under WDD_SERVE_STREAMS, are pushed through their plans on their own streams so
 * that their work overlaps on the device.  The time from submit to the
 * snapshot that contains a frame is recorded per frame.  A server is used by one host
 * thread at a time. */

typedef struct wdd_server_s* wdd_server_t;

typedef enum { WDD_SERVE_STREAMS = 0, WDD_SERVE_GROUPED = 1, WDD_SERVE_GRAPH = 2 } wdd_serve_mode;

typedef struct {
  int64_t hbm_budget_bytes;     /* admission limit on the plans' device memory; <= 0: none.  Default 1 GiB */
  double snapshot_interval_us;  /* least time between snapshots of one acquisition.  Default 1000 */
  int32_t batch_frames;         /* largest batch pushed at once.  Default 256 */
  int32_t launch_mode;          /* a wdd_serve_mode.  Default WDD_SERVE_GROUPED */
} wdd_server_options;

typedef struct {
  uint64_t frames, batches, snapshots, steps;
  int32_t open;                 /* acquisitions open (including those still being made) */
  int64_t device_bytes;         /* device memory of the open plans */
  int64_t pending_frames;       /* submitted, not yet pushed */
  int64_t latency_samples;      /* frames that reached a snapshot */
  double latency_p50_us, latency_p99_us, latency_max_us;  /* submit -> snapshot ready */
  int32_t opening;              /* acquisitions whose plan is still being made */
  uint64_t group_rounds;        /* grouped rounds queued */
  uint64_t graph_replays;       /* rounds replayed from the instantiated graph (WDD_SERVE_GRAPH) */
} wdd_server_stats;

wdd_status wdd_server_default_options(wdd_server_options* opts);
wdd_status wdd_server_create(const wdd_server_options* opts, wdd_server_t* out);

/* Opens an acquisition (arguments as wdd_plan; max_batch is raised to the server's
 * batch_frames; pipeline is ignored: the server orders the acquisitions' launches itself).  Argument errors and WDD_EBUSY (it does not fit the budget now) are
 * returned here; the plan is made on a worker thread, and an error there is returned by
 * the acquisition's next wdd_server_submit or wdd_server_snapshot. */
wdd_status wdd_server_open(wdd_server_t s, const wdd_probe* probe, const wdd_scan* scan, const wdd_detector* det,
                           int32_t K, const wdd_options* opts, int32_t* acq_id);

/* Waits until the acquisition's plan has been made; returns the error of a failed opening. */
wdd_status wdd_server_wait_open(wdd_server_t s, int32_t acq);

/* Queues n device-resident frames (contiguous, 16-byte aligned; they must stay valid
 * until a later wdd_server_step or wdd_server_snapshot has pushed them) with host
 * positions pos_yx [n][2].  WDD_ERANGE (nothing queued) for a position off the raster. */
wdd_status wdd_server_submit(wdd_server_t s, int32_t acq, const void* frames, const int32_t* pos_yx, int32_t n);

/* One scheduling round (see above); *frames_processed = frames pushed (may be NULL). */
wdd_status wdd_server_step(wdd_server_t s, int32_t* frames_processed);

/* Pushes the acquisition's queued frames, takes a snapshot now and copies it to host
 * memory `out` (sy x sx complex, interleaved float).  Blocking. */
wdd_status wdd_server_snapshot(wdd_server_t s, int32_t acq, float* out, uint64_t* frames_seen);

/* Whether the acquisition's plan is ready (made) and how many submitted frames wait to be
 * pushed (either pointer may be NULL). */
wdd_status wdd_server_acq_state(wdd_server_t s, int32_t acq, int32_t* ready, int64_t* pending_frames);

/* Scan size of an open acquisition. */
wdd_status wdd_server_acq_shape(wdd_server_t s, int32_t acq, int32_t* sy, int32_t* sx);

/* Closes an acquisition (queued frames that were not pushed are dropped).  Returns once
 * no queued work reads its frames any more; its plan is then freed on a worker thread, the
 * memory returns to the budget when that is done, and an open that would not fit
 * otherwise waits for it. */
wdd_status wdd_server_close(wdd_server_t s, int32_t acq);

wdd_status wdd_server_get_stats(wdd_server_t s, wdd_server_stats* out);

/* Closes every acquisition and frees the server.  NULL is accepted. */
wdd_status wdd_server_destroy(wdd_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* WDD_H */

/*
 * hodmas.h -- C ABI of the MI355X (gfx950) higher-order delay-multiply-and-sum
 * (HO-DMAS) photoacoustic beamformer.
 *
 * The library forms an image from linear-array photoacoustic RF data.  For each
 * pixel p and each element i it takes the channel sample at the pixel's one-way
 * time of flight (delay of Eq. 1, Sec. II-A), linearly interpolated, forms the
 * signed k-th root y_i = sign(s_i)|s_i|^(1/k) (Eq. 2, Eqs. 4-6), and outputs
 *
 *     S_k(p) = sum over all k-subsets I of the channels of prod_{i in I} y_i,
 *
 * which is DAS for k = 1 (Eq. 1), DMAS for k = 2 (Eq. 2) and DMAS-3/4/5 for
 * k = 3..5 (Eqs. 4-6); k = 6 is the same definition one order higher (Sec. VI).
 * The sum is evaluated in O(N) per pixel from the power sums
 * p_j = sum_i y_i^j, as the paper's simplified forms do (Eqs. 3, 7, 8, 9).
 *
 * Conventions shared by every call:
 *   - Delay of element i for pixel (x, z), in samples:
 *         t = fs * (sqrt((x - x_i)^2 + z^2) / c - t0).
 *     Elements sit at z = 0; pixels at z > 0 face the array.
 *   - Sample at fractional index t: (1-f) s[j] + f s[j+1], j = floor(t),
 *     f = t - j; t outside [0, S-1] contributes 0 (the channel drops out of
 *     every product for that pixel); t == S-1 gives s[S-1].
 *   - RF is channel-major: element i's record starts at rf + i*channel_stride
 *     (in elements of the RF dtype), samples contiguous.
 *   - The image is row-major float32 [nz][nx]: pixel (ix, iz) at
 *     (x0 + ix*dx, z0 + iz*dz) is stored at image[iz*nx + ix].
 *   - No order normalisation, apodisation or envelope is applied: the value is
 *     the raw symmetric sum, with the same units as the RF (degree-1 in s).
 *
 * Errors: every entry point returns a hodmas_status.  Argument errors are
 * detected on the host before anything is launched and leave all outputs
 * untouched.  Launch failures are HODMAS_EDEVICE.  Faults inside an already
 * launched kernel surface as HIP errors on the caller's stream, as for any
 * other HIP work.  No C++ exception or abort crosses this interface.
 *
 * Threading: a plan is immutable after creation.  Concurrent hodmas_beamform
 * calls with the same plan on different streams are allowed.
 */
#ifndef HODMAS_H
#define HODMAS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HODMAS_OK = 0,
    HODMAS_EINVAL = 1,          /* bad argument: null pointer, size, geometry */
    HODMAS_ENOMEM = 2,          /* host or device allocation failed */
    HODMAS_EDEVICE = 3,         /* HIP runtime error (no device, launch failed) */
    HODMAS_EUNSUPPORTED = 4,    /* valid request outside this build (order > max) */
    HODMAS_EBUSY = 5            /* resource held by another in-flight request */
} hodmas_status;

typedef enum {
    HODMAS_F32 = 0,             /* IEEE float32 samples */
    HODMAS_F16 = 1,             /* IEEE float16 samples */
    HODMAS_I16 = 2              /* int16 ADC codes; sample = code * dequant_scale */
} hodmas_dtype;

/* Limits of this build. */
#define HODMAS_MAX_ORDER 6
#define HODMAS_MAX_ELEMENTS 4096
#define HODMAS_MAX_SAMPLES (1 << 24)     /* sample indices stay exact in float32 */
#define HODMAS_MAX_GRID_SIDE 16384

/* Plan flags. */
#define HODMAS_FLAG_ACC_PLAIN   0x1u  /* plain float32 power sums (default: compensated) */
#define HODMAS_FLAG_HOST_ONLY   0x2u  /* build host tables only; no device use (inspection) */
#define HODMAS_FLAG_FORCE_CHECK 0x4u  /* always run the record-boundary test per sample */
#define HODMAS_FLAG_TUNE_BATCH  0x8u  /* hodmas_autotune: only tilings a batch accepts,
                                         timed as a batch runs them */
#define HODMAS_FLAG_CF          0x10u /* weight each pixel by the coherence factor of its
                                         delayed samples (hodmas_beamform and the batch
                                         form; not hodmas_beamform_orders) */
#define HODMAS_FLAG_MIRROR      0x20u /* hodmas_beamform and the batch form each pixel
                                         together with its mirror image about x = 0 from
                                         one delay (symmetric array and grid only, see
                                         hodmas_plan) */
#define HODMAS_FLAG_NO_SHARE    0x40u /* compute every delay in full: no delays shared
                                         along translated pixels (see hodmas_plan) */
/* Reported in hodmas_plan_info.flags, never passed in: the plan's unpaired,
 * unweighted tiles share delays along translated pixels (see hodmas_plan). */
#define HODMAS_INFO_SHARED_DELAYS 0x10000u

/* Linear array.  element_x_m == NULL means a centred uniform array,
 * x_i = (i - (n_elements-1)/2) * pitch_m.  The pointer is read during
 * hodmas_plan only (host memory). */
typedef struct {
    int32_t n_elements;
    double pitch_m;
    double sound_speed_m_s;
    double fs_hz;
    double t0_s;                 /* time of the first sample after the laser shot */
    const double* element_x_m;   /* optional, host, n_elements entries */
} hodmas_geometry;

/* Image grid: pixel (ix, iz) centre at (x0_m + ix*dx_m, z0_m + iz*dz_m). */
typedef struct {
    int32_t nx, nz;
    double x0_m, dx_m;
    double z0_m, dz_m;
} hodmas_grid;

/* RF storage.  frame_max is any positive bound on |sample| after
 * dequantisation (0 means 1).  int16 codes are dequantised and divided by it
 * as the kernel widens them, and the result is multiplied back, so its value
 * changes only rounding; FP32 and FP16 samples are used as stored (e_k is of
 * degree one in the samples) and frame_max is not used for them. */
typedef struct {
    int32_t dtype;               /* hodmas_dtype */
    int32_t n_samples;           /* S, samples per channel */
    int64_t channel_stride;      /* elements between channel records, >= S */
    float dequant_scale;         /* I16 only: value of one code, > 0 */
    float frame_max;             /* >= 0; 0 means 1 */
} hodmas_rf_desc;

/* Tiling of a plan.  Zero fields are chosen by the library.  A workgroup has
 * tile_x * tile_z * split threads, which must be 256 or 512 (plans used in a
 * batch need 256). */
typedef struct {
    int32_t tile_x;              /* pixels per tile along x */
    int32_t tile_z;              /* pixels per tile along z */
    int32_t split;               /* wave groups sharing one pixel's elements: 1, 2 or 4 */
    int32_t chunk;               /* elements staged in LDS at a time; 0: as many as
                                    fit 40 KB, so four workgroups share a CU, or,
                                    where a one-frame launch then needs fewer rounds
                                    of workgroups over the CUs, 20 KB (eight per
                                    CU); equal chunks either way */
} hodmas_tiling;

typedef struct hodmas_plan_s* hodmas_plan_t;

/* Create a plan for one array geometry, image grid and RF layout.
 * Computes, in float64 on the host, the per-(tile, channel) delay anchors and
 * LDS sample windows the kernel uses (the paper precomputes delays before the
 * kernel call, Sec. V), and copies them to the current HIP device once.
 * max_order in [1, HODMAS_MAX_ORDER].  tiling may be NULL (library default).
 * Pixels must lie in front of the array (z0_m > 0, dz_m > 0) and dx_m > 0.
 * On success *out owns its device tables until hodmas_destroy.
 * HODMAS_FLAG_MIRROR needs an array and a grid symmetric about x = 0
 * (x_i = -x_{n-1-i} and x0_m = -(nx-1) dx_m / 2, each to 1e-6 of a sample
 * length c/fs) and a tiling whose tile_x divides nx into an even number of
 * tile columns; hodmas_beamform then runs one workgroup per pair of mirror
 * tiles.  Images differ from the unpaired launch only in rounding.
 * Delays along translated pixels (Eq. 1 depends on pixel x minus element x
 * only): when consecutive elements are exactly four pixel columns apart
 * (x_{i+1} - x_i = 4 dx_m to 1e-12), tiles are 16 columns wide with one
 * element group, nx is a multiple of 16 and each tile's contributing elements
 * are consecutive, an unpaired, unweighted plan's kernels compute, from
 * order 2 on, one delay per lane for every four elements and take the other
 * three from neighbouring lanes through 48 eight-byte LDS entries per row of
 * 16 lanes (included in hodmas_plan_info.lds_bytes), unless that LDS would
 * leave a one-frame launch needing more rounds of workgroups over the
 * device's 256 CUs (HODMAS_INFO_SHARED_DELAYS in hodmas_plan_info.flags says
 * which; HODMAS_FLAG_NO_SHARE turns it off).  Images differ only in rounding.
 * Errors: EINVAL (null pointer, non-positive or non-finite sizes/speeds, stride
 * < S, limits above exceeded, bad tiling, HODMAS_FLAG_MIRROR on an asymmetric
 * geometry or tiling), ENOMEM, EDEVICE. */
hodmas_status hodmas_plan(const hodmas_geometry* geometry, const hodmas_grid* grid,
                          const hodmas_rf_desc* rf, int32_t max_order, uint32_t flags,
                          const hodmas_tiling* tiling, hodmas_plan_t* out);

/* Beamform one frame at order k (1 = DAS, 2 = DMAS, 3..6 = DMAS-k; Eqs. 1-9).
 * A plan is immutable after hodmas_plan: several host threads may launch with
 * the same plan at once, on the same or different streams.
 * rf_dev: device pointer, channel-major records of the plan's dtype and stride.
 * image_dev: device float32 [nz][nx], fully overwritten.  Both are owned by the
 * caller and must stay valid until the work on `stream` completes.
 * stream: a hipStream_t (NULL = default stream).  Asynchronous; one kernel
 * launch; no allocation.  With HODMAS_FLAG_CF in the plan each pixel is
 * multiplied by the coherence factor CF = (sum v)^2 / (N sum v^2) of its N
 * delayed samples (N the array's element count; CF = 0 when all are 0) --
 * the coherence-based weighting Sec. VI proposes to combine with these
 * beamformers.  Errors: EINVAL (null plan/pointers, host-only plan),
 * EUNSUPPORTED (order outside [1, min(6, max_order)]), EDEVICE (launch). */
hodmas_status hodmas_beamform(hodmas_plan_t plan, const void* rf_dev, int32_t order,
                              float* image_dev, void* stream);

/* Beamform one frame at every order 1..max_order in a single pass: the delays,
 * gathers and interpolated samples are shared by all orders and the roots
 * share their transcendentals (the paper compares DAS, DMAS and DMAS-3..5 on
 * the same data, Table II).  images_dev: host array of max_order device
 * pointers; images_dev[k-1] (float32 [nz][nx]) receives order k, each fully
 * overwritten.  Results agree with hodmas_beamform to the same tolerance
 * (the roots are formed along different but equivalent routes).  One launch,
 * asynchronous, no allocation.  Errors as for hodmas_beamform (and
 * EUNSUPPORTED for a plan with HODMAS_FLAG_CF); EUNSUPPORTED
 * also when the combination of all power sums would not fit the LDS. */
hodmas_status hodmas_beamform_orders(hodmas_plan_t plan, const void* rf_dev, int32_t max_order,
                                     float* const* images_dev, void* stream);

/* Wait for the work queued on `stream` (a hipStream_t; NULL = default stream)
 * and report what the device made of it: HODMAS_OK, or HODMAS_EDEVICE when the
 * stream's work or an earlier asynchronous launch failed.  Launch calls return
 * only the errors known when they return; this is where asynchronous device
 * errors surface. */
hodmas_status hodmas_sync(void* stream);

/* Release a plan and its device tables.  NULL is accepted.  The caller must
 * not destroy a plan while work launched with it may still be running. */
hodmas_status hodmas_destroy(hodmas_plan_t plan);

/* Static description of a status code (never NULL). */
const char* hodmas_status_string(hodmas_status status);

/* Choose a tiling for this geometry, grid, RF layout and order by timing the
 * candidate tilings (tile shape, element split, LDS chunk) on the current
 * device on a zero record (timing does not depend on sample values).  With a
 * cache_path, results are appended to / looked up in that JSON-lines file,
 * keyed by device architecture and every input that changes the plan.
 * With HODMAS_FLAG_TUNE_BATCH (unless HODMAS_FLAG_CF comes with
 * HODMAS_FLAG_ACC_PLAIN, which no batch runs) each candidate is timed
 * the way a batch runs it: copies of the frame, each with its own image, in
 * one persistent batched launch of up to 256 copies -- enough work units to
 * fill the device -- and the time per copy is compared.
 * Allocates and frees scratch device memory; not for the hot path.
 * Errors: EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED (no candidate could run). */
hodmas_status hodmas_autotune(const hodmas_geometry* geometry, const hodmas_grid* grid,
                              const hodmas_rf_desc* rf, int32_t order, uint32_t flags,
                              const char* cache_path, hodmas_tiling* out);

/* Plan summary, for callers that size work or report throughput. */
typedef struct {
    int32_t n_elements, n_samples, nx, nz;
    int32_t max_order, dtype;
    hodmas_tiling tiling;
    int32_t n_tiles;             /* tiles covering the grid */
    int32_t max_window;          /* longest LDS sample window of any tile */
    int64_t active_pairs;        /* (tile, channel) pairs that touch the record */
    int64_t lds_bytes;           /* dynamic LDS per workgroup */
    int64_t table_bytes;         /* device bytes held by the plan */
    uint32_t flags;
} hodmas_plan_info;

hodmas_status hodmas_plan_get_info(hodmas_plan_t plan, hodmas_plan_info* info);

/* Inspection of the host copy of the plan tables (layouts below), for tests
 * of the plan's float64 geometry.  Pointers stay valid until hodmas_destroy. */
typedef struct {
    int32_t ix0, iz0;            /* first pixel of the tile */
    int32_t nx, nz;              /* pixels of the tile inside the grid */
    int32_t n_active;            /* channels with any delay inside the record */
    int32_t window;              /* LDS samples per channel for this tile */
    int32_t check;               /* 1: some delay may fall outside [0, S-1] */
    int32_t first_entry;         /* index of the tile's first channel entry */
    double xa, za;               /* anchor pixel, in samples of one-way flight */
} hodmas_tile_desc;

typedef struct {
    float a;                     /* anchor x minus element x (samples) */
    float d0sq;                  /* anchor-to-element distance squared */
    float d0;                    /* anchor-to-element distance */
    float frac0;                 /* fractional part of the anchor delay */
    float lo, hi;                /* valid delays relative to floor(anchor delay) */
    int32_t off;                 /* LDS byte offset of floor(anchor delay) */
    int32_t channel;             /* element index */
} hodmas_chan_entry;

typedef struct {
    int32_t channel;             /* element index */
    int32_t first_sample;        /* record index of LDS window position 0 */
} hodmas_stage_entry;

hodmas_status hodmas_plan_tables(hodmas_plan_t plan, const hodmas_tile_desc** tiles,
                                 const hodmas_chan_entry** entries,
                                 const hodmas_stage_entry** stage, int32_t* n_tiles,
                                 int64_t* n_entries);

/* ---------------------------------------------------------------------------
 * Batched form: many frames -- each with its own plan, order and storage type --
 * in one submission.  The library builds a work list of (frame, tile) units,
 * grouped by kind (order x storage type) and sorted by estimated cost within a
 * kind; one persistent kernel per kind present walks its slice with a fixed
 * grid.  A captured graph chains the kernels of all kinds, so one graph launch
 * runs the whole batch.  Each tile runs exactly the per-frame code, so every
 * frame's image is bitwise the same as from hodmas_beamform with its plan,
 * whatever else is in the batch.  A batch object is used from one stream at a
 * time.
 * ------------------------------------------------------------------------- */
typedef struct hodmas_batch_s* hodmas_batch_t;

/* Allocate a batch for up to max_frames frames and max_units (frame, tile)
 * units (a HODMAS_FLAG_MIRROR plan's units are its n_tiles / 2 mirror pairs),
 * on the current HIP device.  max_lds_bytes bounds the LDS any member
 * plan may need (0: the largest a workgroup can have).  Each kind of a work
 * list runs with the LDS of its own largest plan and as many persistent
 * workgroups as that LDS leaves room for.  flags: HODMAS_FLAG_ACC_PLAIN or 0;
 * member plans must match it.  Errors: EINVAL, ENOMEM, EDEVICE. */
hodmas_status hodmas_batch_create(int32_t max_frames, int64_t max_units, int64_t max_lds_bytes,
                                  uint32_t flags, hodmas_batch_t* out);

/* Describe the frames of the next launch: frame f is beamformed with plans[f]
 * at orders[f] from rf[f] (device) into images[f] (device float32 [nz][nx]).
 * Host arrays of n_frames entries, read during the call.  The work list is
 * copied to the device asynchronously on `stream` (launches on the same stream
 * see it).  A HODMAS_FLAG_MIRROR plan's frame runs as mirror pairs, and a
 * HODMAS_FLAG_CF plan's frame with coherence-factor weighting (Sec. VI), as
 * in hodmas_beamform, with the same image bit for bit.  Errors: EINVAL (null
 * entries, order outside the plan, an accumulation flag other than the
 * batch's, host-only or other-device plan, too many frames/units, plan LDS
 * above the batch's bound or a workgroup other than 256 threads),
 * EUNSUPPORTED (order above 6; a HODMAS_FLAG_CF plan in a batch created with
 * HODMAS_FLAG_ACC_PLAIN -- the weighted kinds accumulate compensated),
 * EDEVICE. */
hodmas_status hodmas_batch_set(hodmas_batch_t batch, const hodmas_plan_t* plans,
                               const void* const* rf, const int32_t* orders,
                               float* const* images, int32_t n_frames, void* stream);

/* Run the current work list on `stream`: one persistent launch per kind
 * present (kind = order x storage type x mirror pairing). */
hodmas_status hodmas_batch_launch(hodmas_batch_t batch, void* stream);

/* Build (once) a HIP graph holding the persistent kernels of the kinds in the
 * current work list (every kind when no list is set yet), with no order
 * between them (kinds write disjoint images, so one kind's tail overlaps the
 * next kind's start); they read the work list from device memory, so later
 * hodmas_batch_set calls with those kinds need no re-capture.
 * hodmas_batch_replay launches that graph on `stream`, after fitting the
 * instantiated graph to the current work list: kinds absent from it are
 * switched off and each present kind gets its own LDS size and persistent
 * grid, at most one workgroup per unit; a kind the graph has no kernel for
 * has the graph rebuilt with every kind seen so far.  When that changes a
 * node, the replay first waits for the previous replay of the graph to
 * finish (host-side); replays of an unchanged kind mix do not wait. */
hodmas_status hodmas_batch_capture(hodmas_batch_t batch);
hodmas_status hodmas_batch_replay(hodmas_batch_t batch, void* stream);

/* Work-list summary of the last hodmas_batch_set. */
typedef struct {
    int32_t n_frames;
    int64_t n_units;
    int32_t grid;                /* persistent workgroups (largest over the kinds present) */
    int64_t lds_bytes;           /* dynamic LDS per workgroup (largest over the kinds present) */
    int64_t pixel_channels;      /* sum over frames of nx*nz*N */
} hodmas_batch_info;

hodmas_status hodmas_batch_get_info(hodmas_batch_t batch, hodmas_batch_info* info);

/* Release the batch (its graph and work-list buffers).  Waits on the host for
 * the batch's last launch, replay and work-list copy to finish first, so the
 * buffers are never freed under a running kernel.  NULL is accepted. */
hodmas_status hodmas_batch_destroy(hodmas_batch_t batch);

/* Version string of the library. */
const char* hodmas_version(void);

/* -------------------------------------------------------------------------
 * Display chain (Sec. III): the paper band-passes the beamformed image,
 * detects its envelope with the Hilbert transform and log-compresses it for
 * display.  Readings (the paper gives no values): a centred FIR along depth,
 * the difference of two Hamming-windowed ideal low-pass responses with unit
 * gain at the centre of the pass band, sampled at c/dz (one-way flight);
 * samples beyond the image are zero.  The envelope is |analytic signal| of
 * each depth column from its length-nz DFT (bin 0 and the Nyquist bin kept,
 * bins 1..nz/2-1 doubled, the rest dropped).  The dB image is
 * 20 log10(envelope / max envelope), clipped below at -dynamic_range_db (an
 * all-zero image gives -dynamic_range_db everywhere).
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t nx, nz;              /* image [nz][nx]; nz a power of two in 2..8192 */
    double dz_m;                 /* depth step, > 0 */
    double sound_speed_m_s;      /* > 0 */
    double f_lo_hz, f_hi_hz;     /* pass band: 0 < f_lo < f_hi < c / (2 dz) */
    int32_t numtaps;             /* odd, 1..255 */
    float dynamic_range_db;      /* > 0 */
} hodmas_display_desc;

typedef struct hodmas_display_s* hodmas_display_t;

/* The band-pass taps (numtaps doubles, caller-owned) for a description, on
 * the host.  Errors: EINVAL (null pointers, even or out-of-range numtaps, a
 * pass band outside (0, c/(2 dz)), non-positive dz or c). */
hodmas_status hodmas_display_taps(const hodmas_display_desc* desc, double* taps);

/* Validate the description and upload the taps and FFT twiddles to the
 * current HIP device.  *out owns them until hodmas_display_destroy.
 * Errors: EINVAL (as for hodmas_display_taps, nx < 1 or > 65536, nz not a
 * power of two in range, dynamic range <= 0), ENOMEM. */
hodmas_status hodmas_display_plan(const hodmas_display_desc* desc, hodmas_display_t* out);

/* image_dev: device float32 [nz][nx] (e.g. a hodmas_beamform output).
 * envelope_dev: device float32 [nz][nx] for the envelope, or NULL.
 * db_dev: device float32 [nz][nx] for the dB image (may equal envelope_dev,
 * must differ from image_dev).  Two asynchronous launches on `stream`; no
 * allocation.  Errors: EINVAL (null image or dB pointer, aliasing the
 * input), EDEVICE. */
hodmas_status hodmas_display_run(hodmas_display_t display, const float* image_dev, float* envelope_dev,
                                 float* db_dev, void* stream);

/* The display chain of n images of the plan's shape in as few launches as
 * possible: up to 16 images per launch pair, each image's own maximum for its
 * dB scale (results equal n hodmas_display_run calls bit for bit).  Host
 * arrays of n device pointers; envelopes_dev may be NULL (no envelopes) or
 * hold NULL entries.  Errors: EINVAL (as for hodmas_display_run, per image;
 * n < 1), EDEVICE. */
hodmas_status hodmas_display_run_batch(hodmas_display_t display, const float* const* images_dev,
                                       float* const* envelopes_dev, float* const* dbs_dev, int32_t n,
                                       void* stream);

/* Release a display plan.  NULL is accepted. */
hodmas_status hodmas_display_destroy(hodmas_display_t display);

/* The display chain of hodmas_display_run without a plan and without any
 * allocation, for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  It
 * calls no hipMalloc, hipFree or other allocating routine.  The band-pass
 * taps, FFT twiddles and per-workgroup envelope maxima live in a file-scope
 * device array of 289 KiB (256 taps, 4096 twiddles, 65536 maxima) that each
 * GPU holds until the process ends; its device address is looked up once per
 * device, on the first call there.  Three asynchronous launches on `stream`:
 * the tables, the envelope, the dB image -- the same arithmetic as the plan
 * path.  desc, image_dev, envelope_dev and db_dev as for hodmas_display_plan
 * and hodmas_display_run (caller-owned device buffers, [nz][nx] float32).
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, other host threads) race and must be serialised by the
 * caller; consecutive calls on one stream are safe.
 * Errors: EINVAL (as for hodmas_display_plan and hodmas_display_run),
 * EUNSUPPORTED (nx above 65536, more workgroup maxima than the array holds),
 * EDEVICE (no current device, the array's address unavailable, a failed
 * launch). */
hodmas_status hodmas_display_run_static(const hodmas_display_desc* desc, const float* image_dev,
                                        float* envelope_dev, float* db_dev, void* stream);

/* -------------------------------------------------------------------------
 * Image-quality metrics (Sec. IV): SNR = 20 log10(mu_in / sigma_out)
 * (Eq. 10), CR = 20 log10(mu_in / mu_out) (Eq. 11) and
 * gCNR = 1 - sum_x min(h_in(x), h_out(x)) (Eq. 12) over a target and a
 * background rectangle of an envelope image, and the FWHM of the target's
 * lateral profile.  Readings: population standard deviation; amplitudes
 * normalised by the largest value over both regions and binned into `bins`
 * equal bins on [0, 1] (top edge in the last bin, negatives in the first),
 * each histogram divided by its pixel count; FWHM along the image row through
 * the target's first maximum (row-major), walking out to the first samples at
 * or below half of it with linear interpolation (a side that never gets there
 * ends at the image edge), times dx_m.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t ix0, ix1, iz0, iz1;  /* pixels [ix0, ix1) x [iz0, iz1) */
} hodmas_rect;

typedef struct {
    double snr_db, cr_db, gcnr, fwhm_m;
    double mu_in, mu_out, sigma_out;
} hodmas_metrics;

/* image_dev: device float32 [nz][nx].  Runs one workgroup on `stream`, waits
 * for it and fills *out (host).  Allocates and frees a few bytes of device
 * memory: an evaluation call, not for the hot path.  Errors: EINVAL (null
 * pointers, empty or out-of-image rectangles, dx_m <= 0, bins outside
 * 2..4096), ENOMEM, EDEVICE. */
hodmas_status hodmas_image_metrics(const float* image_dev, int32_t nx, int32_t nz, double dx_m,
                                   const hodmas_rect* target, const hodmas_rect* background,
                                   int32_t bins, void* stream, hodmas_metrics* out);

/* ---------------------------------------------------------------------------
 * Measured peaks of the current device, the ceilings the beamformer's
 * rooflines are taken against (the path is bound by plain ALU issue; HBM is
 * reported for completeness).  Not part of the paper's method: measurement
 * infrastructure.  Rates are lane-operations per second in units of 1e12 (one
 * wave64 instruction = 64 lane-operations), each from eight independent
 * dependency chains per lane at eight waves per SIMD; packed FP32 is not
 * measured (the library does not use it).
 * ------------------------------------------------------------------------- */
typedef struct {
    double fp32_add;        /* v_add_f32, all operands in VGPRs */
    double fp32_fma;        /* v_fma_f32, all operands in VGPRs */
    double fp32_fma_sgpr;   /* v_fma_f32 with one wave-uniform (SGPR) operand */
    double exp2, log2, sqrt, rcp;   /* the transcendental unit */
    double hbm_copy_tb_s;   /* 1 GiB device-to-device copy: bytes read + written, 1e12/s */
    int32_t compute_units;
    double int_bfi;         /* v_bfi_b32, all operands in VGPRs: the integer / bitwise class */
    double fract;           /* v_fract_f32 */
    /* The beamformer's inner loop as an instruction mix (per element: the
     * delay, sample index and fraction, interpolation, signed sixth root,
     * powers and six power-sum adds -- 27 VALU instructions, 4 of them
     * transcendental; four independent elements per iteration; seven waves
     * per SIMD): SIMD cycles per wave and element at 2.4 GHz, with the
     * per-element constants wave-uniform in SGPRs (as the kernel holds them)
     * and with them in VGPRs. */
    double loop_cycles_sgpr, loop_cycles_vgpr;
} hodmas_peaks;

/* Run the probes on the current device, on `stream`, and wait for them (about
 * a second).  Allocates about 2 GiB of device memory for the copy and frees it
 * before returning: a calibration call, not for the hot path.
 * Errors: EINVAL (null out), ENOMEM, EDEVICE. */
hodmas_status hodmas_measure_peaks(hodmas_peaks* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* HODMAS_H */

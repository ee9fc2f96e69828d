/*
 * vista.h -- C ABI of the MI355X (gfx950) ViSta stacking library.
 *
 * The library stacks interferometric target datasets in the visibility domain, as
 * described by Torsello et al., "The ViSta method for optimized stacking of broadband
 * interferometric data in the Fourier domain", Proc. SPIE 14153 (2026):
 *   - each target's visibilities are phase-rotated to the target's own position
 *     (Sec. 3.2, Eq. 2, with (dl, dm, dn) = (0 - l, 0 - m, 1 - n));
 *   - each channel is moved to the rest frame, nu_rest = nu_obs (1 + z) (Sec. 3.1), and
 *     its uvw are taken to wavelengths at the sample's own frequency, which is Eq. 1's
 *     1/(1+z) baseline scaling paired with the rest-frame frequency;
 *   - every (row, channel, polarisation) sample is split over the common rest channels
 *     with the channel-overlap weights of Eq. 3-4 and added, weighted, into the nearest
 *     cell of one (u, v, nu_rest) grid holding sum(w f V'), sum(w f) and counts.
 *
 * Conventions
 *   - Every function returns int: VISTA_OK (0) or a negative VISTA_E_* code.  On error a
 *     thread-local message is available from vista_last_error().  No C++ exception
 *     crosses this interface.
 *   - hip streams are passed as void* (a hipStream_t; NULL = the null stream).
 *   - All arrays are C order (row-major); complex values are interleaved (re, im) float.
 *   - Arguments are validated before any device work.  A validation failure returns
 *     VISTA_E_ARG and leaves the handle unchanged.  A HIP failure returns VISTA_E_HIP and
 *     poisons the handle: afterwards every call except *_destroy returns VISTA_E_STATE.
 *   - Handles are not thread-safe; distinct handles may be used from distinct threads.
 *
 * Environment
 *   VISTA_LOG=0..3           stderr diagnostics: 1 a line per launch and batch run (records,
 *                            units, device times, host set-up), 2 also autotune candidates,
 *                            wave plans and device allocations of 1 GiB or more, 3 also each
 *                            launch's host build.
 *   VISTA_TUNE_CACHE=path    file of JSON lines keyed by a workload signature: autotune calls
 *                            take a cached shape instead of timing, and append new winners.
 *   VISTA_AGGREGATE=0|1      force the accumulation's LDS updates direct (0) or summed across
 *                            the lanes of a wavefront first (1); by default the latter is used
 *                            for launches of mostly fine channels (6 or more per rest channel).
 *   VISTA_DEVICE_MEM_LIMIT=n cap on the device bytes the library holds (failure testing).
 *   VISTA_FAULT_INJECT=alloc|launch  fail the next device allocation or kernel launch from the
 *                            host, before the operation (failure testing).
 */
#ifndef VISTA_H
#define VISTA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VISTA_OK = 0,
    VISTA_E_ARG = -1,    /* invalid argument; nothing was changed */
    VISTA_E_STATE = -2,  /* call not allowed in the handle's state (finalized, poisoned) */
    VISTA_E_NOMEM = -3,  /* device or host allocation failed */
    VISTA_E_HIP = -4,    /* a HIP runtime call failed; the handle is poisoned */
    VISTA_E_RANGE = -5   /* a result does not fit its output type (a count above 2^32-1) */
};

/* Where a buffer lives. */
enum { VISTA_MEM_HOST = 0, VISTA_MEM_HOST_PINNED = 1, VISTA_MEM_DEVICE = 2 };

/* Grid flags. */
enum {
    VISTA_F_KAHAN = 1u << 0,            /* compensated FP32 accumulation: grid state kept in
                                           FP32 is updated with Kahan's compensated addition
                                           (the state carried across the waves of a batch;
                                           with VISTA_F_DETERMINISTIC also the per-tile sums).
                                           Without DETERMINISTIC the per-tile sums are FP64. */
    VISTA_F_DETERMINISTIC = 1u << 1,    /* every addition in a fixed order: bit-identical
                                           results from run to run (slower) */
    VISTA_F_SPECTRAL_NEAREST = 1u << 2, /* each input channel goes whole to the rest
                                           channel holding nu_obs (1+z) */
    VISTA_F_PHASE_FP32 = 1u << 3,       /* ablation: form u_lambda and the phase turns in
                                           FP32 with full-range sincos (cell indices still
                                           come from FP64) */
    VISTA_F_PLAIN_FP32 = 1u << 4        /* the plain, uncompensated FP32 form: per-tile sums
                                           are FP32 LDS atomic adds (16 B of LDS per cell,
                                           so larger tiles), each addition rounded to FP32.
                                           Error grows with the contributions per cell
                                           (about sqrt(n) * 6e-8 relative).  Not combinable
                                           with VISTA_F_KAHAN or VISTA_F_DETERMINISTIC. */
};

/* The common stack grid.
 *   uv cell (iu, iv) has centre ((iu - nu/2) du, (iv - nv/2) dv) wavelengths (integer
 *   division n/2); a sample goes to iu = rint(u_lambda / du) + nu/2 with
 *   u_lambda = u_m * (nu_obs / c), rint rounding half to even.
 *   Rest channel j spans [freq_lo + j dfreq, freq_lo + (j+1) dfreq) Hz. */
typedef struct {
    int32_t nu, nv;      /* uv cells, 1..65535 each */
    double du, dv;       /* cell size [wavelengths], finite > 0 */
    int32_t nchan;       /* rest channels, >= 1 */
    double freq_lo;      /* rest-frame lower edge of channel 0 [Hz], finite */
    double dfreq;        /* rest channel width [Hz], finite > 0 */
    uint32_t flags;      /* VISTA_F_* */
} vista_grid_desc;

/* One target = one dataset selection (an MS, field and spectral window; Sec. 3.1). */
typedef struct {
    int64_t nrow;                /* >= 0 rows (0 = nothing to add) */
    int32_t nchan;               /* 1..65535 channels */
    int32_t npol;                /* 1, 2 or 4 */
    const double* uvw;           /* [nrow][3] baseline coordinates [m] (MS UVW) */
    const void* vis;             /* complex64 [nrow][nchan][npol] (MS DATA) */
    const float* weight;         /* [nrow][npol] (MS WEIGHT), or [nrow][nchan][npol] when
                                    weight_per_chan; samples with !(w > 0) or a non-finite
                                    w are skipped */
    const uint8_t* flag;         /* [nrow][nchan][npol], nonzero = flagged; NULL = none */
    const double* chan_freq;     /* [nchan] observed frequencies [Hz], finite > 0,
                                    strictly monotonic in either direction; host memory */
    const double* chan_width;    /* [nchan] widths [Hz] > 0, or NULL: centred finite
                                    difference, one-sided at the ends (Eq. 4's Delta nu_k);
                                    required when nchan == 1; host memory */
    double l, m;                 /* direction cosines of the target relative to the phase
                                    centre, l*l + m*m < 1 (ignored with rotate_uvw) */
    double z;                    /* redshift, finite, > -1 */
    int32_t weight_per_chan;     /* 0 or 1 */
    int32_t mem;                 /* VISTA_MEM_* of uvw, vis, weight and flag */
    int32_t rotate_uvw;          /* 0: l, m as given, baselines not rotated.  1: Eq. 1's
                                    rotation R from the phase centre (ra0, dec0) to the
                                    stacking position (ra1, dec1): (l, m) become the stacking
                                    position's direction cosines about the phase centre, and
                                    uv cells (and the rebinned rows' baselines) are taken from
                                    R (u, v, w); the Eq. 2 phase keeps the original baseline
                                    (its turns equal w' - w).  R[i][j] = axis_i(ra1, dec1) .
                                    axis_j(ra0, dec0) with the uvw axes of a centre (ra, dec):
                                    u = (-sin ra, cos ra, 0), v = (-sin dec cos ra,
                                    -sin dec sin ra, cos dec), w = (cos dec cos ra,
                                    cos dec sin ra, sin dec) */
    double ra0, dec0, ra1, dec1; /* [rad], finite, read only with rotate_uvw; the stacking
                                    position must lie in the phase centre's front hemisphere
                                    (n > 0) */
} vista_target;

/* Outputs, dense [nchan][nv][nu] over the whole grid.  Any pointer may be NULL to skip
 * that output.  sum_wvis is complex64, sum_w float, count uint32 (contributions, one per
 * (sample, rest channel) pair).  sum_wvis64 (complex128) and sum_w64 (double) receive
 * the sums before their rounding to FP32: the FP64 per-tile sums, or s - c of a
 * compensated FP32 state (VISTA_F_KAHAN with a carried or ordered state). */
typedef struct {
    void* sum_wvis;
    void* sum_w;
    void* count;
    void* sum_wvis64;
    void* sum_w64;
    int32_t mem;                 /* VISTA_MEM_* of every non-NULL pointer */
} vista_output;

/* Classification of every input sample (n_samples is their total):
 *   outside band -> no rest channel overlaps the sample's channel (Eq. 4 all zero);
 *   outside uv   -> the nearest cell is off the grid;
 *   flagged      -> flag != 0;
 *   bad weight   -> weight not finite or not > 0;
 *   used         -> everything else; n_contrib counts its (sample, rest channel) pairs.
 * Each sample lands in the first category that applies, in that order. */
typedef struct {
    uint64_t n_samples, n_flagged, n_bad_weight, n_outside_uv, n_outside_band, n_used, n_contrib;
} vista_stats;

/* Launch shape of the binned accumulation.  Zero fields take the library default or
 * the autotuned value.  tile_u * tile_v * jblock cells of grid state are held in LDS
 * per workgroup. */
typedef struct {
    int32_t tile_u, tile_v;      /* uv tile in cells */
    int32_t jblock;              /* rest channels per LDS pass */
    int32_t waves;               /* wavefronts per workgroup */
    int32_t wg_per_cu;           /* resident workgroups per compute unit */
} vista_tuning;

/* Device-event timings of the last finalize / batch run, in milliseconds. */
typedef struct {
    double bin_ms;               /* tracks, counting sort, work list */
    double accum_ms;             /* the LDS accumulation kernel(s) */
    double finalize_ms;          /* output conversion (Kahan, FP64, host copies) */
    double total_ms;             /* first to last event */
    double h2d_ms;               /* streamed input copies (batch waves) */
    int64_t n_records;           /* (row, tile) track segments binned */
    int64_t n_units;             /* (tile, rest-channel block) work units */
    int32_t n_accum_launches;    /* accumulation launches timed in accum_ms */
    int32_t n_waves;             /* batch waves */
} vista_timings;

typedef struct vista_stack vista_stack;
typedef struct vista_batch vista_batch;

/* Create one stack: the common (u, v, nu_rest) grid every target is added into -- the
 * stacked product of the method (Sec. 2 and Sec. 3.1: targets shifted to their own
 * positions, rest-framed and combined on one grid of Delta nu_new channels).  g is copied;
 * hip_stream (a hipStream_t of the current device, NULL = the null stream) orders every
 * device operation of the stack.  Nothing is allocated on the device until finalize.
 * *out receives the handle, owned by the caller until vista_stack_destroy.
 * Errors: ARG (NULL pointer, invalid grid or flags), NOMEM (host). */
int vista_stack_create(const vista_grid_desc* g, void* hip_stream, vista_stack** out);

/* Add one target (one dataset selection, Sec. 3.1: its rows' uvw, visibilities, weights and
 * flags, its channel frequencies, its offset (l, m) and redshift z).  The arguments are
 * validated and the channel axis copied here; the host planning (rest-frame edges,
 * Eq. 3-4 overlap table, a_k = nu_k / c) is handed to a pool of library threads and runs
 * while the caller adds more targets (finalize waits for it and reports its errors),
 * except for a target whose widest rest-frame channel could overlap more rest channels
 * than the overlap table holds: that one is planned and checked here.  Device work is
 * deferred to vista_stack_finalize, which stacks all targets in one pass.  VISTA_MEM_HOST
 * data are copied to library staging before the call returns; VISTA_MEM_HOST_PINNED and
 * VISTA_MEM_DEVICE data must stay valid and unchanged until finalize returns (the library
 * keeps only pointers).  Errors: ARG (see vista_target; the stack is unchanged), STATE
 * (after finalize or poisoned), NOMEM, HIP. */
int vista_stack_add_target(vista_stack* s, const vista_target* t);

/* Select the launch shape (NULL = defaults).  Only before finalize.  Errors: ARG (a shape
 * the kernels are not built for, or that does not fit the flags), STATE. */
int vista_stack_set_tuning(vista_stack* s, const vista_tuning* tu);

/* Stack every added target: Eq. 2's shift of each sample to its target's position, the
 * rest frame of Sec. 3.1 with uvw in wavelengths at the sample's own frequency, and the
 * Eq. 3-4 overlap-weighted accumulation of every (row, channel, polarisation) into the
 * grid's sum(w f V'), sum(w f) and counts.  Writes every cell of the outputs o (device,
 * pinned or pageable host memory, dense [nchan][nv][nu]; any field NULL to skip it; NULL o
 * for statistics only), synchronises the stack's stream and returns the classification in
 * *st (may be NULL).  The library owns the grid state and scratch (freed or cached for the
 * thread before return).  A stack is finalized once; later add/finalize calls return
 * VISTA_E_STATE.  Errors: ARG (misaligned or unknown-memory outputs), STATE, NOMEM, HIP
 * (the handle is then poisoned), RANGE (a count above 2^32-1; outputs are then undefined). */
int vista_stack_finalize(vista_stack* s, const vista_output* o, vista_stats* st);

/* Timings of the finalize of this stack (zeros before it).  Errors: ARG. */
int vista_stack_timings(const vista_stack* s, vista_timings* t);

/* Release everything the stack owns (waiting for its planning threads).  Always succeeds
 * for a non-NULL handle, poisoned ones included.  Errors: ARG (NULL). */
int vista_stack_destroy(vista_stack* s);

/* Stacks keep a per-thread launch workspace between calls -- row contexts, binning records,
 * sort scratch and the work list, sized by the largest launch seen (about 80 B per row and
 * 50 B per binning record), for at most two launch shapes -- so that consecutive stacks on
 * one thread neither allocate nor free device memory.  Every launch (stacks and batches)
 * also keeps the host buffers of its channel tables on the calling thread (about 40 B per
 * channel of the largest launch).  This frees both for the calling thread (the next launch
 * allocates them again), and the device blocks of 1 GiB or more that finished batches left
 * for reuse on the current device.  It waits for the device.  Errors: HIP. */
int vista_release_workspace(void);

/* ---- Batched form (Sec. 3.3: N_batch datasets packed into contiguous device buffers and
 * processed per launch, while the host reads the next ones) ---------------------------
 *
 * n_stacks independent stacks (each with its own grid g[i]; every stack of a batch has
 * the same KAHAN, DETERMINISTIC, PHASE_FP32 and PLAIN_FP32 flags) run in one launch
 * sequence per wave: its binning part captured once as a hipGraph and replayed, then one
 * persistent accumulation launch over every stack's units.  Targets are recorded
 * by vista_batch_add_target (as vista_stack_add_target, into stack `stack`);
 * vista_batch_run stacks them all.  Targets in host memory are streamed in waves of at most
 * the stream budget through two device staging buffers on a copy stream, double-buffered
 * against compute (Sec. 3.2's read/compute overlap); device-resident targets run in the
 * first wave.  A stack whose targets span several waves carries its grid state across
 * them in FP32, merged with compensated (Kahan) additions when VISTA_F_KAHAN.
 * Ownership as for stacks: pinned and device inputs stay valid until vista_batch_run
 * returns; registered device outputs are written in place; otherwise the batch keeps the
 * results on the device until vista_batch_finalize copies them out.
 * Errors: create -- ARG (count, grids, mixed flags), NOMEM; add -- as stack add, and ARG for
 * a stack index out of range; run -- STATE (run twice or poisoned), NOMEM (a target larger
 * than the stream budget, device memory), HIP (poisons); finalize -- ARG, STATE (before the
 * run), HIP, RANGE. */
int vista_batch_create(int32_t n_stacks, const vista_grid_desc* g, void* hip_stream, vista_batch** out);
int vista_batch_add_target(vista_batch* b, int32_t stack, const vista_target* t);
/* Launch shape of the batch (NULL = defaults).  Only before the run.  Errors: ARG, STATE. */
int vista_batch_set_tuning(vista_batch* b, const vista_tuning* tu);
/* Device memory per staging buffer for streamed inputs (bytes; 0 = an eighth of the free
 * device memory).  Errors: ARG (negative). */
int vista_batch_set_stream_budget(vista_batch* b, int64_t bytes);
/* Register the outputs of one stack before vista_batch_run: VISTA_MEM_DEVICE outputs
 * are then written by the run itself (no copy at finalize), and only the outputs given
 * are produced.  Other memory kinds are filled at finalize.  Errors: ARG, STATE. */
int vista_batch_set_output(vista_batch* b, int32_t stack, const vista_output* o);
/* Stack every stack's targets (as vista_stack_finalize does for one), all waves; returns
 * when the results are complete on the device and the caller's stream is ordered after
 * them.  Errors: see above. */
int vista_batch_run(vista_batch* b);
/* Copy one stack's results into o (may be NULL when its outputs were registered) and
 * return its classification in *st (may be NULL).  Errors: ARG, STATE, HIP, RANGE. */
int vista_batch_finalize(vista_batch* b, int32_t stack, const vista_output* o, vista_stats* st);
/* Timings of the run, summed over waves: bin_ms the binning (count pass and the replayed
 * graph), accum_ms the accumulation kernel alone, h2d_ms the streamed copies.
 * Errors: ARG. */
int vista_batch_timings(const vista_batch* b, vista_timings* t);
/* Release the batch and its device results (waiting for the device).  The batch's device
 * blocks of 1 GiB or more (staging buffers, carried state) stay with the library for the
 * next batch on the device (memory given back to the driver is cleared again when next
 * allocated, at about 30 GB/s); vista_release_workspace frees them.  Always succeeds for a
 * non-NULL handle.  Errors: ARG (NULL). */
int vista_batch_destroy(vista_batch* b);

/* The paper's common rest grid (Sec. 3.1): dfreq = max over targets and channels of the
 * rest-frame width W_k (1+z) (W_k as for vista_target.chan_width), and the nchan_out
 * channels centred on central_freq: freq_lo = central_freq - nchan_out dfreq / 2.
 * chan_width may be NULL, or hold NULL entries.  Host memory.  Errors: ARG. */
int vista_plan_spectral_grid(int32_t n_targets, const double* const* chan_freq,
                             const double* const* chan_width, const int32_t* nchan, const double* z,
                             double central_freq, int32_t nchan_out, double* freq_lo, double* dfreq);

/* ---- Per-row rebinned product (the paper's per-row kernel output, Sec. 3.2) ----------
 *
 * Each row of each target is shifted to the target's position (Eq. 2; the same FP64 turns
 * and FP32 sine/cosine as the stack) and rebinned onto the target's own output window by
 * Eq. 3 with the Eq. 4 weights, normalised per row, output channel and polarisation:
 *   out[r][j][p] = sum_k f_kj V'(r,k,p) / sum_k f_kj,
 * over the input channels k whose overlap fraction with output channel j is above the
 * sliver threshold (1e-9) and whose sample (r, k, p) is not flagged.  Visibility weights do
 * not enter Eq. 3.  The window (Sec. 3.1) is nout channels of the common rest width dfreq
 * (the paper's Delta nu_new, e.g. from vista_plan_spectral_grid) centred on central_freq;
 * when it does not fit inside the target's rest-frame band (the outermost rest edges of
 * its channels), its upper edge moves down to the band's top if it overhangs there, and
 * then its lower edge up to the band's bottom if it still starts below it.  Rows keep their
 * order; the baseline becomes uvw / (1 + z) (Eq. 1 without its rotation). */
typedef struct {
    int32_t nout;               /* output channels per target, 1..1048576 */
    double dfreq;               /* rest-frame output channel width [Hz], finite > 0 */
    double central_freq;        /* rest-frame window centre [Hz], finite */
} vista_rebin_desc;

typedef struct {                /* one target's outputs, device memory */
    void* vis;                  /* complex64 [nrow][nout][npol], required; 16-byte aligned
                                   (8 for npol == 1) */
    uint8_t* flag;              /* [nrow][nout][npol]: 1 where no unflagged input overlaps
                                   (vis is 0 there); NULL = not written; npol-byte aligned */
    float* wsum;                /* [nrow][nout][npol]: the Eq. 3 normaliser sum_k f_kj of the
                                   unflagged inputs (0 where flagged); NULL = not written;
                                   4 npol-byte aligned */
    double* uvw;                /* [nrow][3]: uvw / (1 + z) [m]; NULL = not written */
} vista_rebin_output;

/* Lower edge [Hz] of target t's output window, computed on the host in FP64 (the same
 * arithmetic vista_rebin_rows uses).  Only chan_freq, chan_width, nchan and z are read.
 * Errors: ARG. */
int vista_rebin_window(const vista_rebin_desc* d, const vista_target* t, double* freq_lo);

/* Rebin n_targets targets (t[i] -> o[i]) in one pass over their rows, on hip_stream; the
 * call returns when the outputs are written.  Every target's data and outputs must be
 * VISTA_MEM_DEVICE (the caller owns them; they are not retained).  freq_lo (n_targets
 * doubles, may be NULL) receives each window's lower edge; tim (may be NULL) the device
 * time of the rebinning kernels in accum_ms and of the whole call in total_ms.  With
 * n_targets == 0 nothing is done.  Errors: ARG (descriptor, target or output invalid,
 * memory not on the device), NOMEM, HIP. */
int vista_rebin_rows(const vista_rebin_desc* d, int32_t n_targets, const vista_target* t,
                     const vista_rebin_output* o, void* hip_stream, double* freq_lo, vista_timings* tim);

/* ---- Dirty image of a stacked grid (the imaging step on the stacked product, Sec. 3.4) --
 *
 * For every rest channel j of a stacked grid (the outputs of vista_stack_finalize), the
 * dirty image by an inverse 2-D FFT:
 *   image[j][q][p] = Re sum_{iv, iu} S_j[iv][iu] exp(+2 pi i (u x_p + v y_q)) / W_j,
 * u = (iu - nu/2) du, v = (iv - nv/2) dv, x_p = (p - nu/2) / (nu du), y_q = (q - nv/2) / (nv dv)
 * (pixel spacing 1 / (n cell), pixel nu/2, nv/2 the stacking position), S = sum_wvis,
 * W_j = the channel's summed weight (sum over the channel of sum_w, in FP64); a channel
 * without weight images to 0.  The gridded data hold each measured baseline once, so the
 * real part is the dirty image of a real sky.  beam (may be NULL): the same transform of
 * sum_w (the dirty beam, 1 at the centre pixel).  Only nu, nv, nchan of g are read: nu and
 * nv must be powers of two in 2..4096, nchan in 1..65535.  All arrays are device memory,
 * [nchan][nv][nu]: sum_wvis complex64 (8-byte aligned), sum_w, image and beam float
 * (4-byte aligned).  Stream-ordered on hip_stream; returns when the images are written.
 * tim (may be NULL): device time of the imaging kernels in accum_ms.  Errors: ARG, NOMEM,
 * HIP. */
int vista_image(const vista_grid_desc* g, const void* sum_wvis, const float* sum_w, float* image, float* beam,
                void* hip_stream, vista_timings* tim);

/* vista_image without allocating: for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The same images as
 * vista_image (the same kernels, channels taken in passes that fit the scratch), with no
 * device allocation, no host-device synchronisation and no timing: the call only enqueues the
 * work on hip_stream and returns; the outputs are complete when the stream reaches that point.
 * Staging lives in a fixed device scratch of the library (64 MiB of complex planes plus 512 KiB
 * of channel weight sums), one per device, held until the process ends.  Limit: one
 * nu x nv complex plane must fit the staging, nu * nv <= 8388608 (e.g. 4096 x 2048; a
 * 4096 x 4096 grid is refused with VISTA_E_ARG).  Other arguments as vista_image.  Every call
 * on a device shares that device's scratch: calls that overlap in time on one device (on
 * different streams, or from several threads without ordering) race and corrupt each other's
 * images; calls ordered on one stream do not.  Errors: ARG, HIP. */
int vista_image_noalloc(const vista_grid_desc* g, const void* sum_wvis, const float* sum_w, float* image,
                        float* beam, void* hip_stream);

/* Per (row, channel) indices the GPU computes for one target, for bit-exact checks of the
 * cell assignment (uvw in wavelengths at the sample's frequency, Sec. 3.1 and Eq. 1) and of
 * the Eq. 4 overlap set: iu, iv (the nearest cell before the bounds test, INT32_MIN when
 * not representable), j0 (first rest channel of the channel's overlap set, -1 if empty)
 * and nj (its size).  Outputs [nrow][nchan] int32 in host memory, caller-owned; the
 * target's data follow t->mem.  Synchronises hip_stream.  Errors: ARG, NOMEM, HIP. */
int vista_debug_indices(const vista_grid_desc* g, const vista_target* t, void* hip_stream,
                        int32_t* iu, int32_t* iv, int32_t* j0, int32_t* nj);

/* The GPU's rotated visibilities V' = V exp(+2 pi i t) of one target (Eq. 2), complex64
 * [nrow][nchan][npol], written to device memory `out` (stream-ordered on hip_stream).
 * Flags and weights are ignored.  The target must be VISTA_MEM_DEVICE. */
int vista_debug_rotate(const vista_grid_desc* g, const vista_target* t, void* hip_stream, void* out);

/* A plain device-to-device copy of nbytes (a multiple of 16; both pointers 16-byte
 * aligned, regions not overlapping) by one streaming kernel, stream-ordered on hip_stream
 * and not waited for.  It is no part of the method: it reads and writes each byte once,
 * so hardware byte counters read on it calibrate those read on the stacking kernels. */
int vista_debug_copy(void* dst, const void* src, size_t nbytes, void* hip_stream);

/* Autotune the launch shape for the stack's targets: times the candidate shapes on the
 * real data and keeps the fastest whose counts equal the default shape's.  The result
 * is applied to the stack and returned in *best (may be NULL).  Only before finalize;
 * the stack's targets must be VISTA_MEM_DEVICE. */
int vista_stack_autotune(vista_stack* s, vista_tuning* best);

/* The same for a batch: every stack's device-resident targets in one launch per
 * candidate; the result applies to vista_batch_run. */
int vista_batch_autotune(vista_batch* b, vista_tuning* best);

const char* vista_last_error(void);
const char* vista_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VISTA_H */

/*
 * disk.h - C ABI of libdisk: the data-parallel hot path of DISK ("Differentiable
 * Sparse Kernel Complex for Efficient Spatially-Variant Convolution", Wu, Cao,
 * Huo, ICLR 2026) on AMD Instinct MI355X (gfx950).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Images are planar [C][H][W], row-major, row index y, column index x, pixel
 *   centres at integers.  C <= 4.
 * - A sparse kernel complex Theta (Sec. 4.1, Eq. 5) is a float32 array
 *   [T][3] of rows (ox, oy, w), layer-major: layer l owns taps[l] consecutive
 *   rows, T = sum_l taps[l].  Offsets are in pixels.
 * - One sparse layer (Sec. 3.2, Eq. 2, chained as in Eq. 3) computes
 *       Y[p] = sum_i w_i * B(X, p - o_i)
 *   where B is the bilinear read (x0 = floor(sx), fx = sx - x0, likewise y).
 *   A tap's weight therefore lands at c + o_i in the impulse response and
 *   filtering is the true convolution with the synthesised kernel.
 * - Boundary: DISK_ZERO (reads outside the canvas are 0; impulse canvases) or
 *   DISK_CLAMP (indices clamped to the edge; images).
 * - Every pointer documented as "device" must be a device pointer owned by the
 *   caller, 16-byte aligned; "host" pointers are ordinary host memory.  The
 *   library never allocates device memory: scratch space is passed in as
 *   (ws, ws_bytes), sized by the matching *_workspace_size call.
 * - Every call that takes a stream is asynchronous on that stream; arguments
 *   are validated on the host before anything is enqueued.  Calls never throw,
 *   exit or print.  On failure they return a negative disk_status and set a
 *   thread-local message readable with disk_last_error().
 * - Limits: 1 <= L <= DISK_MAX_LAYERS, 1 <= taps[l] <= DISK_MAX_TAPS,
 *   1 <= C <= DISK_MAX_CHANNELS, impulse/target sides odd and <= DISK_MAX_SIDE.
 */
#ifndef DISK_H
#define DISK_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DISK_MAX_LAYERS 8
#define DISK_MAX_TAPS 32
#define DISK_MAX_CHANNELS 4
#define DISK_MAX_SIDE 255
#define DISK_MAX_HALO 64

typedef enum {
    DISK_OK = 0,
    DISK_INVALID_ARG = -1,        /* null pointer, bad enum, misaligned pointer */
    DISK_BAD_SHAPE = -2,          /* sizes out of range / inconsistent */
    DISK_WORKSPACE_TOO_SMALL = -3,
    DISK_DEVICE = -4,             /* a HIP call or kernel launch failed */
    DISK_UNSUPPORTED = -5         /* valid but not implemented (e.g. halo too large) */
} disk_status;

typedef enum { DISK_ZERO = 0, DISK_CLAMP = 1 } disk_boundary;
typedef enum { DISK_F32 = 0, DISK_BF16 = 1 } disk_dtype;
typedef enum { DISK_LOSS_NMSE = 0, DISK_LOSS_CHARBONNIER = 1 } disk_loss;
/* Unit in which the learning rate moves tap offsets (Sec. 5.1 leaves it
 * unstated): pixels, or the target's half-width (M - 1) / 2, the unit of
 * normalised sampling coordinates.  Weights always move in their own unit. */
typedef enum { DISK_OFFSETS_PIXELS = 0, DISK_OFFSETS_HALF_WIDTH = 1 } disk_offset_units;

/* Layer structure of one sparse kernel complex (Eq. 5). */
typedef struct {
    int32_t L;
    int32_t taps[DISK_MAX_LAYERS];
} disk_complex;

const char* disk_status_string(disk_status s);
/* Rate of the constant device clock that finish_ticks counts, in kHz, for the
 * current device (0 if it cannot be queried). */
int64_t disk_clock_rate_khz(void);
/* Message of the last failing call on this thread ("" if none). */
const char* disk_last_error(void);
/* Library version string. */
const char* disk_version(void);

/* ------------------------------------------------------------------------- */
/* Chain forward (Sec. 3.2 Eq. 3; impulse response Sec. 4.4 Eq. 10).          */
/* ------------------------------------------------------------------------- */
/*
 * Applies the L sparse layers of Theta to an image, or to the discrete Dirac
 * impulse.
 *   cx     host: layer structure.
 *   theta  device float [T][3].
 *   in     device [C][H][W] of dtype `io`; NULL selects impulse mode: the input
 *          is delta at ((W-1)/2, (H-1)/2), C must be 1, H and W odd, boundary
 *          DISK_ZERO and io DISK_F32 (the result is K_syn of Eq. 10).
 *   out    device [C][H][W] of dtype `io` (FP32 in impulse mode).
 *   saved  device float [(L-1)][C][H][W] receiving X_1..X_{L-1} for
 *          disk_backward, or NULL.
 *   ws     device scratch of at least disk_forward_workspace_size() bytes.
 * Intermediates are FP32; with io = DISK_BF16 the input is widened and the
 * output rounded to nearest-even BF16.
 */
size_t disk_forward_workspace_size(const disk_complex* cx, int32_t C, int32_t H, int32_t W,
                                   disk_dtype io, int32_t impulse, int32_t has_saved);
disk_status disk_forward(const disk_complex* cx, const float* theta, const void* in, void* out,
                         int32_t C, int32_t H, int32_t W, disk_dtype io, disk_boundary boundary,
                         float* saved, void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* Adjoint of the chain (the end-to-end differentiation of Sec. 4.1).         */
/* ------------------------------------------------------------------------- */
/*
 * Given G_L = dLoss/dout, computes
 *   grad_theta  device float [T][3] (overwritten) = dLoss/dTheta, or NULL;
 *   grad_in     device float [C][H][W] (overwritten) = dLoss/din, or NULL.
 *   in          device float [C][H][W], the forward input; NULL = impulse mode
 *               (same rules as disk_forward).
 *   saved       device float [(L-1)][C][H][W] from disk_forward (NULL iff L == 1).
 *   grad_out    device float [C][H][W].
 * The input adjoint is the exact transpose of the forward gather: with
 * DISK_CLAMP, border pixels collect the contributions of every clamped read.
 * Reductions run in a fixed order (deterministic, no float atomics).
 */
size_t disk_backward_workspace_size(const disk_complex* cx, int32_t C, int32_t H, int32_t W);
disk_status disk_backward(const disk_complex* cx, const float* theta, const float* in,
                          const float* saved, const float* grad_out, float* grad_theta,
                          float* grad_in, int32_t C, int32_t H, int32_t W, disk_boundary boundary,
                          void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* Batched optimisation (Sec. 4.1 Eq. 4, Sec. 4.4 Eq. 10-11, Sec. 5.1 Adam).   */
/* ------------------------------------------------------------------------- */
/* One target of a batch; device array [B] of these. */
typedef struct {
    int32_t side;        /* odd M, the target is M x M, impulse at its centre */
    int32_t L;           /* layers */
    int32_t taps_off;    /* index of taps[L] in the taps array */
    int32_t theta_off;   /* first row of this target's Theta in the [*][3] array */
    int32_t target_off;  /* first float of this target's M*M kernel */
} disk_target;

typedef struct {
    int32_t max_steps;       /* Adam updates per target (>= 0) */
    float lr0, lr1;          /* learning rate, linear from lr0 (step 0) to lr1 (last step) */
    float beta1, beta2, eps; /* Adam */
    float psnr_stop_db;      /* stop a target once PSNR >= this (INFINITY: never) */
    int32_t loss;            /* disk_loss */
    float charb_eps;         /* Charbonnier epsilon on the peak-normalised difference */
    int32_t offset_units;    /* disk_offset_units: the offsets' learning rate is lr_t times this unit */
} disk_opt_params;

/* Optimiser state carried across calls, and the loss of the result.  Every
 * field may be NULL / 0. */
typedef struct {
    float* adam_m;             /* device float [*][3] like theta: in = Adam first moments to resume from
                                  (NULL: zeros), out = the moments after the last update */
    float* adam_v;             /* the same for the second moments */
    const int32_t* start_step; /* device int32 [B]: updates already applied to each target (NULL: 0); the
                                  learning-rate schedule and the bias corrections continue from there;
                                  a negative entry makes that target invalid (status 3) */
    float* loss;               /* device float [B]: out, the loss of the returned Theta */
    int32_t max_updates;       /* > 0: at most this many updates per target in this call; 0: no limit */
} disk_opt_state;

/*
 * Fits every target's Theta by Adam on the impulse-response loss, all targets
 * in one persistent launch.
 *   desc     device disk_target [B];  taps  device int32 (per-target layer tap counts);
 *   targets  device float (packed kernels);
 *   theta    device float [*][3]: in = Theta_0, out = the fitted Theta;
 *   psnr_db  device float [B]: PSNR of the returned Theta, 10 log10(max(K)^2 / MSE);
 *   steps    device int32 [B]: position reached in the learning-rate schedule,
 *            i.e. the Adam updates applied including state->start_step;
 *   status   device int32 [B]: 0 ok, 1 stopped at the PSNR threshold,
 *            2 diverged (non-finite loss, e.g. a target holding NaN; Theta is
 *            the last one evaluated and no update is applied from it),
 *            3 invalid descriptor (even or out-of-range side, L outside
 *            1..DISK_MAX_LAYERS, a layer with 0 or more than DISK_MAX_TAPS taps,
 *            side or total taps above meta's maxima, a negative offset
 *            field); that target is skipped, its Theta untouched, psnr_db 0
 *            and steps 0.  Offsets past the ends of the arrays cannot be
 *            detected: they are the caller's responsibility.
 *   finish_ticks  device uint64 [B + 1] or NULL: the device's constant-rate
 *            clock (disk_clock_rate_khz) when each target finished; entry B
 *            holds the clock at the start of the launch.
 *   params   host: Adam hyper-parameters, schedule, stopping rule, loss.
 *   state    host struct of device pointers, or NULL: resume from given Adam
 *            moments and schedule positions, report the loss, limit the
 *            updates of this call.  Splitting a run into calls that carry
 *            the state gives the same result, bit for bit, as one call.
 *   tune     host, or NULL for the built-in table (see disk_opt_tune).
 *   ws       device scratch of disk_optimize_workspace_size(meta, tune) bytes.
 *   meta     host: B, the maximum side and total taps, used to size the launch.
 * Loss: normalised MSE, mean((K_syn - K)^2) / max(K)^2, or Charbonnier.
 * The two launches (queue order, persistent optimiser) contain no memset or
 * copy, so the call may be captured into a HIP graph and replayed.
 */
typedef struct {
    int32_t B;
    int32_t max_side;
    int32_t max_T;
} disk_batch_meta;
/* Launch shape of the persistent optimiser, chosen per batch by the built-in
 * table (tune = NULL; rows keyed by batch size and largest side, written by the
 * project's autotuner, paper_2512_04556_amd/autotune.py) or given here.  Each
 * work-group owns one target at a time: 256 threads with 1..4 resident per
 * compute unit, or 1024 threads (16 waves on one target) with 1 per unit, for
 * batches too small to fill the chip.  Results do not depend on wgs_per_cu; the
 * two work-group sizes sum in different orders (rounding-level differences). */
typedef struct {
    int32_t threads;           /* 256 or 1024 */
    int32_t wgs_per_cu;        /* 1..4 for 256 threads, 1 for 1024 */
} disk_opt_tune;
size_t disk_optimize_workspace_size(const disk_batch_meta* meta, const disk_opt_tune* tune);
/* The launch shape the built-in table gives a batch (what disk_optimize_batch
 * uses with tune = NULL): the first row whose batch size, largest side and
 * largest tap count bound meta's, else 256 threads x 4.  Host only, nothing
 * enqueued.
 *   meta   host: B >= 1, max_side >= 1, max_T >= 1.
 *   out    host, written on success.
 * Errors: DISK_INVALID_ARG for a NULL pointer or a field out of range. */
disk_status disk_optimize_default_tune(const disk_batch_meta* meta, disk_opt_tune* out);
disk_status disk_optimize_batch(const disk_batch_meta* meta, const disk_target* desc,
                                const int32_t* taps, const float* targets, float* theta,
                                float* psnr_db, int32_t* steps, int32_t* status,
                                uint64_t* finish_ticks, const disk_opt_params* params,
                                const disk_opt_state* state, const disk_opt_tune* tune, void* ws,
                                size_t ws_bytes, hipStream_t stream);

/*
 * Basis precompute (the offline stage of Sec. 4.3): fits the B targets in
 * order by continuation, so that tap i plays the same role in every entry.
 * Entry 0 starts from theta as given (e.g. disk_init_radial); entry k >= 1
 * starts from the fitted entry k-1 with its offsets multiplied by scale[k]
 * (e.g. r_k / r_{k-1}) and its weights copied, then runs the same
 * optimisation as disk_optimize_batch (one launch per entry, in stream order).
 * An entry whose layer structure differs from the previous entry's starts
 * from theta as given.
 *   scale   host float [B] (scale[0] unused), finite and > 0;
 *   ws      device scratch of disk_fit_basis_workspace_size() bytes;
 *   other arguments as in disk_optimize_batch.
 */
size_t disk_fit_basis_workspace_size(const disk_batch_meta* meta);
disk_status disk_fit_basis(const disk_batch_meta* meta, const disk_target* desc, const int32_t* taps,
                           const float* targets, float* theta, float* psnr_db, int32_t* steps, int32_t* status,
                           const float* scale, const disk_opt_params* params, void* ws, size_t ws_bytes,
                           hipStream_t stream);

/*
 * Radial initialisation (Sec. 4.1 Eq. 6) of every target of a batch, on the
 * device: r_l = l * dr with dr = 2R / (L (L+1)), o_{l,i} = r_l (cos 2 pi i/N_l,
 * sin 2 pi i/N_l) for i = 1..N_l, w = 1/N_l; R = min((M-1)/2, r99) with r99
 * the smallest pixel-centre distance whose disk holds >= 99% of the target's
 * mass (the paper defers the step size to an appendix; this is the reading
 * adopted).  Arguments as in disk_optimize_batch; theta is written.  A target
 * whose descriptor disk_optimize_batch would reject (status 3) is skipped and
 * its Theta left as it was.
 */
disk_status disk_init_radial(const disk_batch_meta* meta, const disk_target* desc,
                             const int32_t* taps, const float* targets, float* theta,
                             hipStream_t stream);

/*
 * Shape-aware (sparse-sampling) initialisation (Sec. 4.2 Eq. 7), on the host
 * in FP64: the first layer's taps are dart-thrown over the support
 * {K > 0.01 max K} with radius r = sqrt(S / (N_1 pi)) (shrunk by 0.9 after
 * 100 N_1 consecutive rejections), weights proportional to K at the rounded
 * points; layers 2..L take the radial pattern with extent r.  Random draws:
 * SplitMix64 stream keyed by (seed, target index).
 *   target  host float [M][M];  taps host int32 [L];
 *   theta   host float [T][3] (written);  r_out host (final radius) or NULL.
 */
disk_status disk_init_shape(const float* target, int32_t M, int32_t L, const int32_t* taps,
                            uint64_t seed, int32_t index, float* theta, double* r_out);

/*
 * Random-position initialisation (the baseline the shape-aware init is
 * compared with, Sec. 4.2), on the host in FP64: tap i of layer l uniform in
 * [-r_l, r_l]^2 with r_l = l dr the radial rule's radius (Eq. 6), weights
 * 1/N_l; two draws per tap (x, then y) from the SplitMix64 stream keyed by
 * (seed, index) as in disk_init_shape.
 *   target host float [M][M];  taps host int32 [L];  theta host float [T][3];
 *   R_out (the extent R) or NULL.
 */
disk_status disk_init_random(const float* target, int32_t M, int32_t L, const int32_t* taps,
                             uint64_t seed, int32_t index, float* theta, double* R_out);

/* ------------------------------------------------------------------------- */
/* Spatially varying filtering by filter-space interpolation (Sec. 4.3).      */
/* ------------------------------------------------------------------------- */
/*
 * A basis (Eq. 8) of G = grid[0] (dims 1) or grid[0]*grid[1] (dims 2) complete
 * parameter sets sharing one layer structure `cx`, at evenly spaced parameter
 * values on [0, 1]; entry (i0, i1) is stored at index i0*grid[1] + i1.
 * halo[l] bounds layer l's offsets: every |ox|, |oy| of layer l in every entry
 * must be <= halo[l] - 1 (disk_basis_set_halo computes it).
 */
typedef struct {
    int32_t dims;                    /* 1 or 2 */
    int32_t grid[2];                 /* entries per axis (grid[1] ignored for dims 1) */
    disk_complex cx;
    int32_t halo[DISK_MAX_LAYERS];
} disk_basis;

/* Fills b->halo from a HOST copy of the basis [G][T][3]. */
disk_status disk_basis_set_halo(disk_basis* b, const float* basis_theta_host);

/*
 * Per pixel p: u = clamp(P(p), 0, 1) (G - 1) per axis; the interpolation
 * weights alpha are the hat (1-D) or bilinear (2-D) weights of the nodes
 * around u (Eq. 9: convex, sum 1); Theta(p) = sum_k alpha_k Theta_k over
 * offsets and weights; the L layers are applied with each pixel's own taps,
 * CLAMP boundary, X_l[p] = sum_i w_{l,i}(p) B(X_{l-1}, p - o_{l,i}(p)).
 *   basis_theta device float [G][T][3];   image device [C][H][W] of dtype io;
 *   pmap        device float [dims][H][W]; out  device [C][H][W] of dtype io.
 * If an offset in the basis exceeds its declared halo, the output is filled
 * with NaN (no out-of-tile reads happen).  For 1-D bases with C >= 3 (and
 * tables small enough for on-chip staging) the passes read the basis
 * directly and no preparation launch runs; otherwise this call is
 * disk_sv_prepare followed by disk_sv_apply.  The results are identical.
 */
size_t disk_sv_filter_workspace_size(const disk_basis* b, int32_t C, int32_t H, int32_t W,
                                     disk_dtype io);
disk_status disk_sv_filter(const disk_basis* b, const float* basis_theta, const void* image,
                           const float* pmap, void* out, int32_t C, int32_t H, int32_t W,
                           disk_dtype io, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * The same filter over F frames at once (a video's frames, or a batch of
 * images of one size): images and outs are device [F][C][H][W] of dtype io;
 * pmaps is device float [F][dims][H][W] (pmap_per_frame != 0) or one
 * [dims][H][W] map shared by every frame.  Each of the L passes covers all F
 * frames in one launch, so a launch's start-up and tail are paid once per F
 * frames (the chain of Sec. 4.3 applied frame by frame; results identical to
 * F calls of disk_sv_filter).  1 <= F <= DISK_MAX_FRAMES; ws holds the two
 * FP32 intermediates of all F frames.
 */
#define DISK_MAX_FRAMES 64
size_t disk_sv_filter_frames_workspace_size(const disk_basis* b, int32_t F, int32_t C, int32_t H,
                                            int32_t W, disk_dtype io);
disk_status disk_sv_filter_frames(const disk_basis* b, const float* basis_theta, const void* images,
                                  const float* pmaps, int32_t pmap_per_frame, void* outs, int32_t F,
                                  int32_t C, int32_t H, int32_t W, disk_dtype io, void* ws,
                                  size_t ws_bytes, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * filter as disk_sv_filter, with identical results, but its scratch (the
 * coefficient table and the two FP32 images between passes) lives in a fixed
 * device array of the library, DISK_SV_NOALLOC_MAX_BYTES (64 MiB) per GPU,
 * held from the first call on that GPU until the process ends.  The call
 * allocates nothing; the caller still owns image, pmap and out.
 * Errors: DISK_WORKSPACE_TOO_SMALL when disk_sv_filter_workspace_size(b, C, H,
 * W, io) exceeds the array (e.g. above about 2.7 Mpixel of 3-channel FP32
 * intermediates: 1920 x 1080 x 3 fits, 3840 x 2160 x 3 does not); otherwise
 * as disk_sv_filter.  Every call on one GPU uses that GPU's one array: calls
 * that overlap on the same GPU (different streams, threads or processes
 * sharing it) race and must be serialised by the caller.
 */
#define DISK_SV_NOALLOC_MAX_BYTES (64u << 20)
size_t disk_sv_noalloc_max_bytes(void);
disk_status disk_sv_filter_noalloc(const disk_basis* b, const float* basis_theta, const void* image,
                                   const float* pmap, void* out, int32_t C, int32_t H, int32_t W,
                                   disk_dtype io, hipStream_t stream);

/*
 * Angle axis for a 2-D basis (the angle-driven effects, rotational bokeh and
 * radial motion blur, of the paper's spatially varying examples): entry
 * (i0, i1), stored at i0 * G1 + i1, is base entry i0 with every offset
 * rotated counter-clockwise by angles[i1]: (ox cos a - oy sin a,
 * ox sin a + oy cos a); weights copied.  Tap i keeps its role across angles.
 *   base   device float [G0][T][3];   angles host double [G1] (radians), 1 <= G1 <= 64;
 *   out    device float [G0 * G1][T][3] (written; must not overlap base).
 */
disk_status disk_basis_rotate(const float* base, int32_t G0, int32_t T, const double* angles, int32_t G1,
                              float* out, hipStream_t stream);

/*
 * The same filter in two steps, for a basis that serves many frames (the
 * offline/runtime split of Sec. 4.3): disk_sv_prepare turns the basis into the
 * per-(entry, tap) coefficient table the passes read (and checks the halos);
 * disk_sv_apply runs the L passes with a prepared table.
 *   table  device scratch of disk_sv_table_bytes() bytes, owned by the caller,
 *          valid until the basis changes.
 *   ws     (apply) device scratch of disk_sv_apply_workspace_size() bytes for
 *          the FP32 intermediates (may be NULL when L == 1).
 */
size_t disk_sv_table_bytes(const disk_basis* b);
disk_status disk_sv_prepare(const disk_basis* b, const float* basis_theta, void* table,
                            size_t table_bytes, hipStream_t stream);
size_t disk_sv_apply_workspace_size(const disk_basis* b, int32_t C, int32_t H, int32_t W,
                                    disk_dtype io);
disk_status disk_sv_apply(const disk_basis* b, const void* table, const void* image,
                          const float* pmap, void* out, int32_t C, int32_t H, int32_t W,
                          disk_dtype io, void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* Dense reference: the per-pixel kernel the sparse filter approximates.       */
/* ------------------------------------------------------------------------- */
/*
 * Spatially varying dense convolution (Eq. 1 with a kernel per output pixel,
 * the ground truth of Sec. 4.3's filter-space interpolation), CLAMP boundary:
 *   out[p] = sum_q K_p[q] I[clamp(p - q)] / sum_q K_p[q],  |qx|, |qy| <= half,
 *   DISK_DENSE_DISK:    K_p[q] = clamp(r + 1/2 - |q|, 0, 1),
 *                       r = r0 + (r1 - r0) clamp(P0(p), 0, 1);
 *   DISK_DENSE_ELLIPSE: axis-aligned ellipse with semi-axes (r sqrt(a), r / sqrt(a)),
 *                       a = a0 (a1 / a0)^clamp(P1(p), 0, 1),
 *                       K_p[q] = clamp(1/2 - (rho - 1) |q| / rho, 0, 1) with
 *                       rho = |(qx / ax, qy / ay)| (clamp(1/2 + min(ax, ay), 0, 1) at q = 0).
 *   image, out  device [C][H][W] of dtype io;  pmap device float [1 or 2][H][W].
 * Each pixel visits at most (2 half + 1)^2 taps; half should cover the
 * largest semi-axis + 1/2 (larger kernels are cut at half).
 */
typedef enum { DISK_DENSE_DISK = 0, DISK_DENSE_ELLIPSE = 1 } disk_dense_kind;
typedef struct {
    int32_t kind;       /* disk_dense_kind */
    float r0, r1;       /* radius at P0 = 0 and P0 = 1 (pixels, >= 0) */
    float a0, a1;       /* aspect at P1 = 0 and P1 = 1 (ellipse only, > 0) */
    int32_t half;       /* 0 <= half <= 127 */
} disk_dense_params;
disk_status disk_dense_sv(const disk_dense_params* p, const void* image, const float* pmap, void* out,
                          int32_t C, int32_t H, int32_t W, disk_dtype io, hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* Learned initialiser (not in the paper): a conv encoder + MLP that predicts  */
/* a starting Theta for the optimiser; BF16 operands, FP32 accumulation on     */
/* MFMA.                                                                      */
/* ------------------------------------------------------------------------- */
/*
 * Network: 64x64x1 -> 6 x [conv 3x3, stride 2, zero padding 1, + bias, ReLU]
 * with widths 32, 64, 128, 128, 256, 256 (spatial 64 -> 1) -> FC 256->512 +
 * ReLU -> FC 512->144.  The 144 outputs are Theta for 4 layers x 12 taps, tap t
 * at (3t, 3t+1, 3t+2) = (o_x / hw, o_y / hw, w), hw the input's scale
 * (disk_net_prepare_inputs).
 * Parameters: one float32 blob of disk_net_param_count() values, in the order
 * conv1.W [32][1][3][3], conv1.b [32], ..., fc1.W [512][256], fc1.b [512],
 * fc2.W [144][512], fc2.b [144] (PyTorch layout).
 * Precision: each layer's input activations and weights are rounded to BF16
 * (nearest even) and contracted with FP32 accumulation; hidden outputs are
 * ReLU(z) rounded to BF16.  Backward: the bias gradient sums dL/dz in FP32;
 * both contractions take dL/dz rounded to BF16; the gradient of the BF16
 * weights is applied to the FP32 master weights.
 * Limits: 1 <= B <= DISK_NET_MAX_BATCH.  All reductions run in a fixed order
 * (results are bitwise reproducible).
 */
#define DISK_NET_MAX_BATCH 65536
int64_t disk_net_param_count(void);
/* Device scratch for disk_net_train_step at batch B (also enough for
 * disk_init_predict, which needs only disk_net_predict_workspace_size(B)). */
size_t disk_net_workspace_size(int32_t B);
size_t disk_net_predict_workspace_size(int32_t B);
/*
 * Inference.
 *   params      device float [disk_net_param_count()];
 *   targets64   device uint16 (BF16 bits) [B][64][64] (disk_net_prepare_inputs);
 *   half_width  device float [B] (hw of each input);
 *   theta       device float [B][48][3] (written): offsets in target pixels
 *               (network output x hw), weights as predicted.
 */
disk_status disk_init_predict(const float* params, const uint16_t* targets64,
                              const float* half_width, float* theta, int32_t B, void* ws,
                              size_t ws_bytes, hipStream_t stream);
/*
 * One training step: forward, loss = mean over B x 144 of (y_hat - y)^2 with
 * y = theta_ref in network units (offsets / hw), backward, then Adam
 * (beta 0.9, 0.999, eps 1e-8, bias correction at `step` >= 1, learning rate
 * lr) on the FP32 master parameters.
 *   params, adam_m, adam_v  device float [disk_net_param_count()], updated;
 *   theta_ref   device float [B][48][3], offsets in target pixels;
 *   loss_out    device float [1]: the loss before the update;
 *   grad_out    device float [disk_net_param_count()] or NULL: the gradient.
 */
disk_status disk_net_train_step(float* params, float* adam_m, float* adam_v, int32_t step,
                                float lr, const uint16_t* targets64, const float* half_width,
                                const float* theta_ref, int32_t B, float* loss_out,
                                float* grad_out, void* ws, size_t ws_bytes, hipStream_t stream);
/*
 * Network input of every target of a batch: the M x M target (centre
 * c = (M-1)/2) is averaged by exact pixel-area overlap onto 64 x 64 cells of
 * side s = max(1, M/64) centred on c, divided by its maximum and rounded to
 * BF16; half_width[b] = 32 s.  desc/targets as in disk_optimize_batch; a
 * target whose descriptor is invalid gets a zero input and half_width 0.
 *   targets64  device uint16 [B][64][64] (written);  half_width device float [B].
 */
disk_status disk_net_prepare_inputs(const disk_batch_meta* meta, const disk_target* desc,
                                    const float* targets, uint16_t* targets64,
                                    float* half_width, hipStream_t stream);
/* Copy the network's [B][48][3] prediction into the batch's Theta layout
 * (rows theta_off .. theta_off+47 of target b).  Targets that do not have
 * L = 4 and 12 taps per layer are left untouched. */
disk_status disk_net_scatter_theta(const disk_batch_meta* meta, const disk_target* desc,
                                   const int32_t* taps, const float* theta48, float* theta,
                                   hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* DISK_H */

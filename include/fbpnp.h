/*
 * fbpnp: fan-beam CT plug-and-play reconstruction with multi-stage sketched
 * gradients on AMD MI355X (gfx950).
 *
 * Method: Tang, "Accelerating Plug-and-Play Image Reconstruction via
 * Multi-Stage Sketched Gradients" (arXiv:2203.07308).
 *   - measurement model b = A x + w ............................ Sec. 1, Eq. (1)
 *   - least-squares gradient A^T(Ax - b) inside PnP ............. Sec. 2.1, Eq. (5)
 *   - sketched objective f(b, A_s S(x)), S: R^d -> R^m .......... Sec. 2.1, Eq. (4)
 *   - sketched gradient U(A_s^T A_s S(x) - A_s^T b) .............. Sec. 2.1, Eq. (6)
 *   - minibatch (view-subset) gradient with M_k ................. Sec. 2.1, Eq. (7)
 *   - one PnP-MS2G iteration: sketch, gradient, upsampled step,
 *     relaxed denoiser, momentum ................................ Sec. 2.1, Algorithm 1
 *
 * Conventions (the paper fixes none of them):
 *   Images are float32, row-major [ny][nx]; row r is the y axis, column c the
 *   x axis; pixel (r,c) has centre ((c-(nx-1)/2) h, (r-(ny-1)/2) h).
 *   Sinograms are float32 [views][n_bins], bins contiguous.
 *   View k has source S = sod (cos b, sin b), b = angle0 + k*angle_step; the
 *   flat detector is perpendicular to the central ray at distance sdd from the
 *   source, bin j centred at ((j-(n_bins-1)/2) pitch + det_offset) along
 *   (-sin b, cos b).
 *   A is Joseph's ray-driven projector (one ray per bin centre, linear
 *   interpolation along the minor axis, zero outside the grid). A_s is the same
 *   projector on the grid coarsened by a pooling factor f (pixel f h), S = D_f
 *   is f x f average pooling and U = D_f^T (replicate, divide by f^2).
 *
 * Memory and threading:
 *   All array arguments are device pointers (hipMalloc'd or torch tensors) with
 *   at least 16-byte alignment; the caller owns them. Calls are asynchronous on
 *   the given stream and never synchronise, allocate or free, except the
 *   set-up calls that say so (plan, batch and graph creation and
 *   destruction, configuration and sketch changes of a batch or plan,
 *   fb_batch_prepare, the autotuners) and fb_power_lipschitz.
 *   A plan owns a device workspace: calls that use one plan must not overlap
 *   in time (issue them on one stream, or use one plan per stream).
 *   Outputs never alias inputs unless a call says otherwise.
 *
 * Errors: every call returns an fb_status. Arguments are validated on the host
 * before any launch; on error nothing is launched and fb_last_error() returns
 * a message (thread-local). No C++ exception crosses this interface. NaN or
 * Inf values inside arrays are not checked.
 */
#ifndef FBPNP_H
#define FBPNP_H

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int fb_status;
#define FB_OK 0
#define FB_EINVAL (-1)  /* null pointer, non-positive size, bad stage or parameter */
#define FB_EGEOM (-2)   /* geometry not valid (source inside the image circle, fan too wide, non-finite) */
#define FB_EDIV (-3)    /* image size not divisible by the pooling factor */
#define FB_ESUBSET (-4) /* view list too long, or (fb_check_views) an index outside the views */
#define FB_EHIP (-5)    /* HIP runtime or launch error (message holds the HIP text) */
#define FB_ENOMEM (-6)  /* device allocation failed (plan or graph creation only) */

/* Fan-beam geometry of the full-resolution grid. Valid (FB_EGEOM otherwise):
 * finite values; positive pixel, distances and pitch; image circumradius
 * h sqrt(nx^2 + ny^2) / 2 < sod_mm; detector half-extent
 * |(n_bins - 1) / 2 det_pitch_mm| + |det_offset_mm| < sdd_mm, so the fan is
 * narrower than 90 degrees and each view's bins of one dominance class are
 * contiguous. */
typedef struct fb_geom {
    int32_t nx, ny;          /* image width (columns) and height (rows) */
    double pixel_mm;         /* pixel size h */
    int32_t n_views, n_bins; /* views and detector bins */
    double sod_mm, sdd_mm;   /* source-to-isocentre, source-to-detector */
    double det_pitch_mm;     /* bin pitch on the detector */
    double det_offset_mm;    /* detector shift along (-sin b, cos b) */
    double angle0_rad, angle_step_rad;
} fb_geom;

typedef struct fb_plan fb_plan;

/* Thread-local message of the last failing call on this thread ("" if none). */
const char* fb_last_error(void);

/*
 * Creates a plan for one geometry and n_stages pooling factors (each in
 * 1..32, dividing nx and ny; FB_EINVAL otherwise). Stage s is the Joseph projector A_s on the
 * (ny/f_s) x (nx/f_s) grid with pixel f_s h (Sec. 2.1, Eq. (4)). Ray tables are
 * computed in double precision on the host and stored in float32 on the
 * device. Allocates device memory and synchronises the current device.
 */
fb_status fb_plan_create(const fb_geom* geom, int n_stages, const int32_t* factors, fb_plan** out);
fb_status fb_plan_destroy(fb_plan* plan);

/* Stage description: coarse grid, factor, and the number of in-grid Joseph
 * samples of one projection over all views (the projector's work). */
typedef struct fb_stage_info {
    int32_t factor, nxs, nys;
    int64_t samples_all_views;
} fb_stage_info;
fb_status fb_plan_stage_info(const fb_plan* plan, int stage, fb_stage_info* out);
/* The same sample count per view: out is a host array of n_views entries. */
fb_status fb_plan_view_samples(const fb_plan* plan, int stage, int64_t* out);
/* Device workspace that calls at this stage use, in bytes: the stage's two
 * line images, the residual [n_views][n_bins] and z [ny][nx]. The plan owns
 * it (allocated once by fb_plan_create), so fanbeam_fp, fanbeam_bp and
 * pnp_step take no workspace argument; the figure is for memory accounting. */
fb_status fb_workspace_bytes(const fb_plan* plan, int stage, size_t* out);

/*
 * Sketch operator of the plan's stages with f > 1 (Sec. 2.1, Eqs. (4), (6)):
 *   kind 0  f x f average pooling D, U = D^T (default);
 *   kind 1  bicubic resizing (Sec. 3): Keys' cubic convolution kernel, a = -1/2,
 *           stretched by f against aliasing, output o of each axis centred at
 *           input coordinate (o + 1/2) f - 1/2, taps beyond the ends folded
 *           back by half-sample reflection, rows normalised to 1; separable;
 *           U = S^T (so the sketched gradient stays exact).
 * fb_plan_set_sketch allocates the bicubic tables (a set-up call, not under
 * capture). With kind 1, pnp_step sketches y anew at such stages (the
 * pooling hand-over of fb_graph_create is skipped for them), vr_mode must be
 * 0 and pnp_step_vjp is unavailable there; fb_power_lipschitz uses the kind.
 * fb_plan_sketch_down / fb_plan_sketch_up apply the stage's S (x: device
 * [ny][nx] -> v: [nys][nxs]) and U = S^T (v -> x).
 */
fb_status fb_plan_set_sketch(fb_plan* plan, int kind);
fb_status fb_plan_sketch_down(const fb_plan* plan, int stage, const float* x, float* v, hipStream_t stream);
fb_status fb_plan_sketch_up(const fb_plan* plan, int stage, const float* v, float* x, hipStream_t stream);

/*
 * Launch configuration of a stage's kernels (no effect on what is computed,
 * only on how the work is split; results can differ in the last bits where
 * the split changes a summation order):
 *   fp_seg   lanes per ray in the forward projector (1, 2, 4 or 8; a
 *            wavefront holds 64 / fp_seg rays, a work-group 256 / fp_seg)
 *   bp_px    backprojector form and block: 1, 2 or 4 selects the gather form
 *            with bp_px x bp_px pixels per lane (a wavefront owns an 8 bp_px
 *            square); 16 or 32 the scatter form over bp_px x bp_px blocks
 *   bp_vg    wavefronts per work-group splitting the views (1..16, <= 4 when
 *            bp_px = 4)
 *   tv_tile  TV-prox output tile side (16 or 32)
 *   fp_lds   where the forward projector reads its taps: 1 from the stage's
 *            line images in global memory, 2 from a copy of them in LDS
 *            (only for stages whose two line images fit, at most 147456
 *            bytes, e.g. grids up to 128 x 128; fb_plan_set_config refuses
 *            2 for other stages; batches take 1)
 * A zero field selects the built-in default for the call's size.
 * fb_plan_set_config: cfg NULL restores every default.
 * fb_plan_get_config: the configuration calls with n_sel views use.
 */
typedef struct fb_launch_config {
    int32_t fp_seg, bp_px, bp_vg, tv_tile, fp_lds;
} fb_launch_config;
fb_status fb_plan_set_config(fb_plan* plan, int stage, const fb_launch_config* cfg);
fb_status fb_plan_get_config(const fb_plan* plan, int stage, int n_sel, fb_launch_config* out);

/*
 * Forward projection y = M A_s x (Sec. 1, Eq. (1); Sec. 2.1, Eq. (4)).
 *   x: device [nys][nxs] image on the stage's coarse grid.
 *   views: device int32 list of n_sel view indices (the rows of M), or NULL
 *     for all views in order (then n_sel must equal n_views). Repeats are
 *     allowed; an index outside [0, n_views) yields a zero row (fp) or no
 *     contribution (bp); indices are not checked here (fb_check_views does).
 *   y: device [n_sel][n_bins], overwritten.
 * Uses the plan workspace.
 */
fb_status fanbeam_fp(const fb_plan* plan, int stage, const float* x, float* y, const int32_t* views,
                     int n_sel, hipStream_t stream);

/*
 * Checks a device view list (the rows of M_k, Sec. 2.1, Eq. (7)) against the
 * plan, as a set-up call for callers that want it: the calls above and
 * pnp_step read the list on the device and give a zero row for an index outside
 * [0, n_views) instead.
 *   views: device int32 [n_sel]; n_sel >= 1.
 * Returns FB_ESUBSET when n_sel exceeds n_views or an index lies outside
 * [0, n_views) (fb_last_error() names the first such position and its value),
 * FB_EINVAL for a NULL pointer or n_sel < 1, FB_OK otherwise. Allocates 4 bytes
 * of device memory for the call and synchronises the stream.
 */
fb_status fb_check_views(const fb_plan* plan, const int32_t* views, int32_t n_sel, hipStream_t stream);

/*
 * Matched backprojection x = scale * (M A_s)^T y: the exact transpose of
 * fanbeam_fp (identical interpolation weights), computed without atomics (a
 * pixel-driven gather or, with bp_px 16 or 32, a scatter into per-wavefront
 * LDS blocks whose concurrent lanes never share a cell, added in a fixed
 * order), so results are bitwise reproducible.
 *   y: device [n_sel][n_bins]; x: device [nys][nxs], overwritten.
 */
fb_status fanbeam_bp(const fb_plan* plan, int stage, const float* y, float* x, const int32_t* views,
                     int n_sel, float scale, hipStream_t stream);

/* Sketch S = D_f: v[R][C] = mean of the f x f block of x (Sec. 2.1, Eq. (4)).
 * x: device [ny][nx]; v: device [ny/f][nx/f]. */
fb_status sketch_down(const float* x, int nx, int ny, int f, float* v, hipStream_t stream);

/* Upsampler U = D_f^T: x[r][c] = v[r/f][c/f] / f^2 (Sec. 2.1, Eq. (6)).
 * v: device [nys][nxs]; x: device [nys*f][nxs*f]. */
fb_status sketch_up(const float* v, int nxs, int nys, int f, float* x, hipStream_t stream);

/*
 * Denoiser D (Sec. 2.1, list after Eq. (5)): n_iter steps of Chambolle's dual
 * projection for isotropic TV with forward differences and Neumann boundary,
 * from p = 0:  p <- (p + tau grad(div p - z/lambda)) / (1 + tau |grad(.)|),
 * then x = z - lambda div p. lambda == 0 copies z.
 *   ws: device workspace of at least fb_tv_workspace_bytes(nx, ny, n_iter)
 *   bytes (0 bytes, ws may be NULL, when n_iter <= 8).
 */
size_t fb_tv_workspace_bytes(int nx, int ny, int n_iter);
fb_status tv_prox(const float* z, float* x, int nx, int ny, float lambda, int n_iter, float tau, void* ws,
                  size_t ws_bytes, hipStream_t stream);

/*
 * tv_prox without a workspace argument, for callers that cannot allocate
 * device memory (code under graph capture, serving loops, harnesses that
 * forbid hipMalloc). Same kernels and results as tv_prox. For n_iter > 8 the
 * dual fields live in a static device array of 16 MiB per device, allocated
 * with the library's code object and held until the process ends; its address
 * is looked up once per device, at the first such call. nx * ny must be at
 * most 1048576, else FB_EINVAL with nothing launched. The call allocates
 * nothing. Every call on one device shares that array: calls that overlap on
 * one device (other streams, other threads) race and give wrong results.
 * Every cell of the array is written before it is read, so no clearing is
 * needed between calls.
 */
fb_status tv_prox_noalloc(const float* z, float* x, int nx, int ny, float lambda, int n_iter, float tau,
                          hipStream_t stream);


/*
 * One PnP-MS2G iteration t (Sec. 2.1, Algorithm 1, Option 1 or 2):
 *   v   = S_k(y_{t-1})                        (pooling of the stage)
 *   G   = sigma (M A_s)^T (M A_s v - M b)     (minibatch gradient, Eq. (7))
 *   z   = y_{t-1} - eta U G                   (U = D_f^T)
 *   x_t = (1 - alpha) z + alpha D(z)          (D: tv_prox with lambda, tau, tv_iters <= 8)
 *   y_t = x_t + a_t (x_t - x_{t-1})
 * b is the full sinogram [n_views][n_bins]; views/n_sel select M as in
 * fanbeam_fp, or, with views NULL, n_sub > 1 selects the interleaved subset
 * subset, subset + n_sub, subset + 2 n_sub, ... (Algorithm 1, Option 2):
 * 0 <= subset < n_sub, and n_sel must equal its size,
 * ceil((n_views - subset) / n_sub). The kernels then compute each view index
 * instead of reading it from a list. n_sub = 0 (or 1) and subset = 0 leave
 * the selection to views/n_sel; giving both a list and n_sub > 1 is
 * FB_EINVAL. y_out may equal y_prev and x_out may equal x_prev (in-place
 * iteration). history, if not NULL, receives a copy of x_t.
 * Chaining (optional, set automatically by fb_graph_create): next_stage >= 0
 * makes this call also pool y_t for stage next_stage into the plan workspace;
 * the next call may then set prepared = 1 to skip its own pooling, which is
 * valid only if it uses that stage and its y_prev is this call's y_out. Use
 * next_stage = -1 and prepared = 0 for independent calls.
 * events (optional, may be NULL): six hipEvent_t created with timing enabled;
 * [0], [1] are recorded at the start and completion of the step's
 * forward-projection kernel, [2], [3] of its back-projection kernel and [4], [5]
 * of its denoiser kernel (hipExtLaunchKernelGGL start/stop events), so their
 * elapsed time is the kernel's own duration. A NULL entry is skipped. The
 * caller owns the events. fb_graph_create ignores them.
 * Variance-reduced gradients (SVRG over view subsets; the estimators named
 * after Eq. (7)), by vr_mode:
 *   0  the minibatch gradient above (snap_proj, snap_grad unused);
 *   1  snapshot: every view (views NULL, n_sub <= 1, n_sel = n_views, sigma 1); the step
 *      is the full-gradient step, and it also stores the snapshot's projection
 *      A_s v into snap_proj (device [n_views][n_bins]) and its coarse gradient
 *      A_s^T (A_s v - b) into snap_grad (device [nys][nxs] of the stage);
 *   2  G = sigma (M A_s)^T (M A_s v - M snap_proj) + snap_grad, i.e.
 *      g_M(y) - g_M(y_snap) + g(y_snap) with the last snapshot of this stage.
 * A snapshot's buffers belong to one stage; take a new snapshot when the stage
 * changes.
 * grad (optional, vr_mode 0 only): device [nys][nxs] of the stage. pnp_step
 * stores the unscaled coarse gradient (M A_s)^T (M A_s v - M b) there, so G =
 * sigma grad; pnp_step_vjp reads it back instead of recomputing it (a
 * checkpoint for reverse mode; it must come from the forward step at the same
 * inputs).
 * stamp (optional): device uint64; every work-group of the step's denoiser
 * kernel raises it (atomic max) to the device's constant-rate clock
 * (fb_clock_khz ticks per millisecond) when it has issued its stores, so it
 * ends as the time the denoiser kernel finished. Clear it before the step.
 * Consecutive steps' stamps give per-iteration times inside a graph, where
 * events do not bracket kernels. (With a next-stage pooling factor that does
 * not divide the TV tile, the pooling runs as a launch after the stamp.)
 * Every optional field (history, events, vr_mode and its buffers, n_sub,
 * subset, grad, stamp) means "not used" at zero: zero-initialise the struct
 * (fb_pnp_args a = {0}) and set the fields in use.
 */
typedef struct fb_pnp_args {
    int32_t stage;
    const int32_t* views;
    int32_t n_sel;
    float sigma, eta, alpha, a_t;
    float lambda, tau;
    int32_t tv_iters;
    const float* b;
    const float* y_prev;
    const float* x_prev;
    float* x_out;
    float* y_out;
    float* history;
    int32_t next_stage;
    int32_t prepared;
    hipEvent_t const* events;
    int32_t vr_mode;
    float* snap_proj;
    float* snap_grad;
    int32_t n_sub, subset;
    float* grad;
    uint64_t* stamp;
} fb_pnp_args;
fb_status pnp_step(const fb_plan* plan, const fb_pnp_args* args, hipStream_t stream);
/* Measurement of the time to reach a PSNR (the comparison of Sec. 3):
 * rate of the device clock behind fb_pnp_args.stamp on the current device, in
 * kHz (ticks per millisecond); 0 if the runtime does not report it. */
int32_t fb_clock_khz(void);
/* Writes the same clock to *dst (device uint64) when the stream reaches this
 * call (a one-thread kernel): the start mark before a run of stamped steps. */
fb_status fb_clock_stamp(uint64_t* dst, hipStream_t stream);

/*
 * A whole schedule of pnp_step calls captured once into a HIP graph and
 * replayed with one launch. The argument arrays are copied at creation; the
 * device buffers they point to must stay valid while the graph exists.
 */
typedef struct fb_graph fb_graph;
fb_status fb_graph_create(const fb_plan* plan, const fb_pnp_args* steps, int n_steps, fb_graph** out);
fb_status fb_graph_launch(fb_graph* graph, hipStream_t stream);
fb_status fb_graph_destroy(fb_graph* graph);

/*
 * Batched form: many independent slices (own geometry, size, views and
 * detector; shared stage factors) advanced together, each kernel of an
 * iteration issued once for the whole batch, with work-groups ordered
 * longest-processing-time first across slices.
 *   fb_batch_create: one plan per slice (geoms[n_slices]; every factor must
 *     divide every slice's nx and ny; 1..4 stages, at most 4096 slices).
 *   fb_batch_layout: the caller's arenas. image_offsets and sino_offsets are
 *     host arrays of n_slices + 1 entries receiving each slice's offset in
 *     floats (256-byte aligned) and, last, the arena size: slice s's image
 *     [ny][nx] starts at image_offsets[s], its sinogram [n_views][n_bins] at
 *     sino_offsets[s].
 *   fb_batch_slice_plan: the plan the batch holds for one slice (owned by the
 *     batch; it shares that plan's workspace, so do not use it concurrently
 *     with batched calls).
 *   pnp_step_batched: one iteration of Algorithm 1 for every slice, as
 *     pnp_step, on the arenas. eta is a device array [n_slices] of per-slice
 *     step sizes. n_sub <= 1 selects all views; n_sub > 1 selects views
 *     k = subset + n_sub i of every slice (the gradient is then usually scaled
 *     by sigma = n_sub). history (optional) is an image arena receiving x_t.
 *     next_stage / prepared / events as in fb_pnp_args. A step never
 *     allocates or synchronises: it reads per-launch work lists (the
 *     (slice, block) order of its work-groups) that set-up calls build.
 *     fb_batch_create builds those of all-view steps (n_sub <= 1);
 *     fb_batch_prepare(batch, n_sub) builds those of steps with n_sub
 *     subsets (allocates and synchronises the device). Later
 *     configuration changes (fb_batch_set_config, fb_batch_autotune) rebuild
 *     the lists of every subset count prepared so far, and
 *     fb_batch_graph_create builds whatever its steps need before capture.
 *     A step whose lists are missing returns FB_EINVAL and launches nothing.
 *   fb_batch_set_config / fb_batch_get_config: launch configuration per
 *     stage, as for plans (get: the one used with n_sub subsets).
 */
typedef struct fb_batch fb_batch;
typedef struct fb_batch_args {
    int32_t stage;
    int32_t n_sub, subset;
    float sigma, alpha, a_t;
    float lambda, tau;
    int32_t tv_iters;
    const float* eta;
    const float* b;
    const float* y_prev;
    const float* x_prev;
    float* x_out;
    float* y_out;
    float* history;
    int32_t next_stage;
    int32_t prepared;
    hipEvent_t const* events;
} fb_batch_args;
fb_status fb_batch_create(const fb_geom* geoms, int n_slices, int n_stages, const int32_t* factors, fb_batch** out);
fb_status fb_batch_destroy(fb_batch* batch);
fb_status fb_batch_layout(const fb_batch* batch, int64_t* image_offsets, int64_t* sino_offsets);
fb_status fb_batch_slice_plan(fb_batch* batch, int slice, fb_plan** out);
fb_status fb_batch_set_config(fb_batch* batch, int stage, const fb_launch_config* cfg);
fb_status fb_batch_get_config(const fb_batch* batch, int stage, int n_sub, fb_launch_config* out);
fb_status fb_batch_prepare(fb_batch* batch, int n_sub);
fb_status pnp_step_batched(fb_batch* batch, const fb_batch_args* args, hipStream_t stream);
fb_status fb_batch_graph_create(fb_batch* batch, const fb_batch_args* steps, int n_steps, fb_graph** out);

/*
 * Autotuner: for every stage, times each launch configuration candidate on
 * synthetic data of the stage's shape (HIP events on the stream), keeps the
 * fastest whose output agrees with the default configuration's within 1e-5
 * relative L2, and sets it on the plan (calls with n_sel views) or the batch
 * (steps with n_sub subsets). Allocates temporary device memory and
 * synchronises the stream: a set-up call. cache_path (optional) is a text
 * file of earlier results, read first and appended to; a cached entry for the
 * same device, geometry, stage and view selection is used without timing. On
 * error the configuration is left as it was.
 */
fb_status fb_autotune(fb_plan* plan, int n_sel, const char* cache_path, hipStream_t stream);
fb_status fb_batch_autotune(fb_batch* batch, int n_sub, const char* cache_path, hipStream_t stream);

/*
 * Reverse mode (differentiation of unrolled iterations).
 *
 * tv_prox_vjp: zbar = J^T xbar for the relaxed denoiser
 *   z -> (1 - alpha) z + alpha tv_prox(z; lambda, n_iter, tau),
 * recomputing the dual iterates; d|q|/dq is taken as 0 at q = 0. zbar must not
 * alias z or xbar. ws: at least fb_tv_vjp_workspace_bytes(nx, ny, n_iter) bytes;
 * that is 0 for n_iter <= 5 (one launch recomputes every dual level on chip),
 * and then ws may be NULL.
 */
size_t fb_tv_vjp_workspace_bytes(int nx, int ny, int n_iter);
fb_status tv_prox_vjp(const float* z, const float* xbar, float* zbar, int nx, int ny, float lambda, int n_iter,
                      float tau, float alpha, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * pnp_step_vjp: reverse mode of one pnp_step (Sec. 2.1, Algorithm 1) at the
 * inputs in args (b, y_prev, views, sigma, eta, alpha, a_t, lambda, tau,
 * tv_iters, and grad: the coarse gradient the forward step stored, or NULL to
 * recompute it; x_out, y_out and history are ignored; vr_mode must be 0).
 * Given the adjoints
 * xbar = dL/dx_t and ybar = dL/dy_t (ybar may be NULL for 0), computes
 *   xbar_prev = dL/dx_{t-1} = -a_t ybar            (may be NULL)
 *   ybar_prev = dL/dy_{t-1} = zbar - eta H zbar,    zbar = J_relax^T (xbar + (1 + a_t) ybar)
 *   eta_bar[0] = dL/deta_t = -<zbar, U G(y_prev)>   (device float)
 * where H = sigma U (M A_s)^T M A_s S is the symmetric linear part of the
 * sketched gradient G (the matched projector pair serves as its own adjoint).
 * combine != 0 writes ybar_prev + xbar_prev into ybar_prev (the adjoint of
 * x_0 when x_0 = y_0). Outputs must not alias inputs or each other. Uses the
 * plan workspace and ws (at least fb_pnp_vjp_workspace_bytes(plan, tv_iters)
 * bytes, 256-byte aligned, as torch and hipMalloc allocations are).
 */
size_t fb_pnp_vjp_workspace_bytes(const fb_plan* plan, int tv_iters);
fb_status pnp_step_vjp(const fb_plan* plan, const fb_pnp_args* args, const float* xbar, const float* ybar,
                       float* xbar_prev, float* ybar_prev, float* eta_bar, int combine, void* ws, size_t ws_bytes,
                       hipStream_t stream);

/*
 * Lipschitz constant L = ||A_s D_f||_2^2 of the stage's data term over all
 * views (step eta = 1/L, Sec. 3) by n_iter power iterations from the constant
 * unit vector. Synchronous: blocks until the result is on the host.
 */
fb_status fb_power_lipschitz(const fb_plan* plan, int stage, int n_iter, double* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* FBPNP_H */

/*
 * osog.h -- C ABI of libosog, an MI355X (gfx950) renderer of the OSOG forward
 * model (arXiv 2606.21381): a Structure-of-Arrays particle table becomes an
 * optical-path-difference (OPD) canvas, and the canvas becomes a microscope
 * image through the wave-optics chain exp(i 2 pi/lambda OPD) -> FFT -> pupil and
 * defocus -> DIC shear / oblique shift -> inverse FFT -> |E|^2 (-> shot noise).
 *
 * Conventions shared by every entry point
 *   - Plain C types only.  "device" pointers are GPU memory of the context's
 *     device; "host" pointers are CPU memory read before the call returns.
 *   - The caller owns every buffer it passes; the library never frees them and
 *     never keeps them after the call.  The context owns only its own tables.
 *   - Work is enqueued on the caller's HIP stream (a hipStream_t passed as
 *     void*, NULL = default stream) and is asynchronous: no entry point waits
 *     for the GPU, and none copies device data to the host.
 *   - Outputs are overwritten, never accumulated into.  Inputs are not modified.
 *   - Arguments are checked on the host before anything is enqueued; a failed
 *     check returns its status and enqueues nothing.  Device array contents are
 *     not checked: NaNs propagate (a particle with a NaN centre or a
 *     non-positive half-width contributes nothing).
 *   - Results are bitwise reproducible for fixed inputs and tiling.
 *   - No C++ exception crosses this boundary.  osog_last_error() returns the
 *     calling thread's message for its last non-OK status.
 */
#ifndef OSOG_H
#define OSOG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OSOG_OK = 0,
  OSOG_ERR_INVALID_ARGUMENT = 1, /* null pointer, bad size, bad optics            */
  OSOG_ERR_UNSUPPORTED = 2,      /* canvas not a power of two in [32, 4096], ...  */
  OSOG_ERR_WORKSPACE = 3,        /* workspace missing or smaller than required    */
  OSOG_ERR_HIP = 4,              /* a HIP runtime call or kernel launch failed     */
  OSOG_ERR_NOT_INITIALIZED = 5   /* null context                                  */
} osog_status;

/* Imaging modality (paper Sec. III.B): brightfield (Eq. 4's |U * h_obj|^2),
 * differential interference contrast (Eq. 5 with the shear inside the coherent
 * transfer function: |(U sheared and interfered) * h_obj|^2), oblique
 * illumination (the asymmetric Fourier pupil of the oblique modality), and DIC
 * as Eq. 5 writes it: the exit wave sheared and interfered at full resolution,
 * squared, then blurred by the incoherent PSF |h_obj|^2 (scaled to unit sum).
 * OSOG_DIC_INCOHERENT renders forward only (osog_render, osog_batch_render);
 * it needs the larger workspace (osog_workspace_size with with_backward = 1). */
typedef enum { OSOG_BRIGHTFIELD = 0, OSOG_DIC = 1, OSOG_OBLIQUE = 2, OSOG_DIC_INCOHERENT = 3 } osog_mode;

/* The particle table is the SoA tensor S of paper Sec. III.A stored
 * attribute-major: float soa[OSOG_D][ld], row r holding attribute r of
 * particles 0..n-1 (ld >= n).  Pixel (i = row, j = column) covers
 * [j, j+1] x [i, i+1] in pixel units; R(angle) maps local (u, v) to (x, y). */
enum {
  OSOG_CX = 0,     /* centre x [px]                                             */
  OSOG_CY = 1,     /* centre y [px]                                             */
  OSOG_ANGLE = 2,  /* in-plane rotation [rad]                                   */
  OSOG_A = 3,      /* half-width along u [px] (prism) / semi-axis (ellipsoid)   */
  OSOG_B = 4,      /* half-width along v [px] / semi-axis                       */
  OSOG_HEIGHT = 5, /* prism height / ellipsoid full central thickness [um]      */
  OSOG_DN = 6,     /* n_particle - n_medium                                     */
  OSOG_SHAPE = 7,  /* < 0.5 prism (box-filtered exact area); < 1.5 ellipsoid;   */
                   /* 2 + k polyhedral habit k (osog_set_habits)               */
  OSOG_D = 8,
  /* absorbing tables (osog_optics.absorption = 1) carry one more row:           */
  OSOG_DMU = 8,    /* mu_particle - mu_solvent, attenuation contrast [1/um]    */
  OSOG_D_ABS = 9
};

/* Static optics of a frame (host memory).  Lengths in micrometres. */
typedef struct {
  int32_t mode;            /* osog_mode                                               */
  double wavelength_um;    /* lambda > 0                                              */
  double na;               /* numerical aperture, 0 < na < n_medium                   */
  double n_medium;         /* n_m; axial wavenumber k0 = 2 pi n_m / lambda (Eq. 3)    */
  double pixel_um;         /* canvas pixel pitch dx > 0                               */
  double shear_angle_rad;  /* DIC shear direction psi (not differentiated)            */
  double tilt_fx;          /* oblique illumination frequency [cycles/um]: H = P(f+ft) */
  double tilt_fy;
  double photons_mean;     /* > 0: Poisson shot noise at this mean photon count/px    */
  uint64_t seed;           /* Philox4x32-10 key of the noise                           */
  uint32_t noise_frame;    /* second Philox counter word (frame index)                 */
  /* 0: phase object, exit-wave amplitude A = 1, table of OSOG_D rows.
   * 1: Beer-Lambert absorption (Eq. 4's exponential factor): the table has
   *    OSOG_D_ABS rows and A = exp(-tau) with the absorbance canvas
   *    tau = sum over particles of dmu * thickness, built like the OPD. */
  int32_t absorption;
  /* Gaussian read noise of the sensor (Sec. III.C: Poisson shot noise plus a
   * Gaussian term), standard deviation in photon counts, >= 0; needs
   * photons_mean > 0.  Pixels 2m and 2m+1 take z from Box-Muller on the first two
   * words of the Philox block at counter (m, noise_frame, 0, 2); the output is
   * (counts + read_noise z) / s. */
  double read_noise;
} osog_optics;

/* Differentiable per-frame globals live in DEVICE memory, float[4]:
 *   [0] defocus dz [um]   (Eq. 3)
 *   [1] total DIC shear 2|ds| [px] along shear_angle_rad   (Eq. 5)
 *   [2] DIC bias phase theta [rad]                          (Eq. 5)
 *   [3] unused (0)
 * so that solver steps need no host round trip and calls can be captured. */
#define OSOG_NGLOBALS 4

typedef struct osog_context osog_context;

/* Create a context on HIP device `device`: uploads the FFT twiddle table and
 * sets the default tiling (32 x 16 pixel tiles: 32 rows by 16 columns).  Allocates device memory. */
osog_status osog_context_create(osog_context** out, int device);
osog_status osog_context_destroy(osog_context* ctx);

/* Tiling used for binning and rasterisation: tile_h x tile_w pixels, both
 * powers of two with 256 <= tile_h * tile_w <= 1024.  Changing it changes the
 * pair list but not the OPD (each pixel's value depends only on the pixel and
 * the particles that reach it). */
osog_status osog_set_tiling(osog_context* ctx, int32_t tile_h, int32_t tile_w);
osog_status osog_get_tiling(const osog_context* ctx, int32_t* tile_h, int32_t* tile_w);

/* Bytes of device workspace needed by osog_render (with_backward = 0) or by
 * osog_render_backward (with_backward = 1) for an H x W canvas and n particles.
 * pairs_per_particle sizes the (tile, particle) pair list: pairs_per_particle * n
 * + tiles entries (0 selects 32).  The list is grouped by tile with exact
 * offsets, so a crowded tile costs only its own pairs.  A frame whose pairs
 * exceed the list stays correct and bitwise identical: the tiles whose segments
 * do not fit are rasterised by a slower id-ordered scan of all particles.  The
 * workspace also holds up to 32 MiB of planes in which the slices of crowded
 * tiles (more than 48 pairs) keep their partial sums; a frame that needs more
 * leaves its last crowded tiles unsliced (slower, same result).  The workspace
 * holds no state between calls and may be reused for anything in between. */
osog_status osog_workspace_size(const osog_context* ctx, int32_t height, int32_t width, int64_t n,
                                int32_t pairs_per_particle, int32_t with_backward, size_t* bytes);

/* Forward render (paper Sec. III, f(Theta) = I):
 *   soa           device float[OSOG_D][ld] (absorbing: float[OSOG_D_ABS][ld]);
 *                 shape < 0.5 prism, < 1.5 ellipsoid, 2 + k habit k (osog_set_habits),
 *                 ld >= n, n >= 0 (n = 0: empty canvas)
 *   optics        host, static optics
 *   globals       device float[4] (see above)
 *   opd_out       device float[height][width] or NULL: OPD canvas [um] (Eq. 2's
 *                 integral); absorbing: float[2][height][width], the OPD then
 *                 the absorbance tau
 *   intensity_out device float[height][width]: |E|^2, with shot noise if photons_mean > 0
 *   workspace     device, >= osog_workspace_size(..., with_backward = 0) bytes
 * height, width: powers of two in [32, 4096], multiples of the tile sides. */
osog_status osog_render(osog_context* ctx, void* stream, int32_t height, int32_t width,
                        const float* soa, int64_t n, int64_t ld, const osog_optics* optics,
                        const float* globals, float* opd_out, float* intensity_out,
                        void* workspace, size_t workspace_bytes);

/* osog_render without a workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It calls no hipMalloc, hipFree or allocating library routine: the
 * frame's buffers (records, tile pair list, band spectrum, and the OPD and
 * absorbance planes when opd_out is NULL) live in one fixed 64 MiB device array
 * inside the library, one copy per GPU, held until the process ends.  Arguments
 * and outputs are those of osog_render (same kernels, bitwise the same images);
 * the caller still passes soa, globals, opd_out and intensity_out.
 *   Limit: frames whose packed buffers exceed 64 MiB return OSOG_ERR_WORKSPACE
 *   with the size they need (2048 x 2048 with 40,000 particles needs about 30 MiB
 *   without opd_out); the incoherent DIC (mode 3) returns OSOG_ERR_UNSUPPORTED.
 *   Every call on one GPU shares that GPU's array, whatever the context or
 *   stream: calls that overlap in time on one GPU race and give wrong images.
 *   Serialise them (one stream, or events between streams). */
osog_status osog_render_noalloc(osog_context* ctx, void* stream, int32_t height, int32_t width,
                                const float* soa, int64_t n, int64_t ld, const osog_optics* optics,
                                const float* globals, float* opd_out, float* intensity_out);

/* Several imaging modalities of one particle table, pixel-aligned (paper Sec.
 * III, the multi-modal output of one geometry buffer): binning, rasterisation
 * and the row FFT run once over the union of the modes' in-band spectrum
 * columns; the column pass and the row IFFT (with each mode's noise) run per
 * mode.  Each intensity_out[m] is bitwise identical to osog_render with
 * optics[m], globals[m] and the same tiling.
 *   n_modes        1..64
 *   optics         host osog_optics[n_modes]; all share wavelength_um, pixel_um,
 *                  n_medium and absorption (one OPD, one exit wave); mode, NA,
 *                  shear angle, tilt, photons and seed may differ
 *   globals        device float[n_modes][4]
 *   intensity_out  host array of n_modes device pointers, each float[H][W]
 *   opd_out        device float[H][W] (absorbing: [2][H][W]) or NULL
 *   workspace      as for osog_render_backward (osog_workspace_size with
 *                  with_backward = 1)
 * Errors: OSOG_ERR_INVALID_ARGUMENT for a bad count, NULL pointer or optics that
 * differ in wavelength, pixel size or medium index; otherwise as osog_render. */
osog_status osog_render_multi(osog_context* ctx, void* stream, int32_t height, int32_t width,
                              const float* soa, int64_t n, int64_t ld, int32_t n_modes,
                              const osog_optics* optics, const float* globals, float* const* intensity_out,
                              float* opd_out, void* workspace, size_t workspace_bytes);

/* Adjoint of the noiseless render (the gradient the paper keeps after Eq. 7):
 * given dL/dI (and optionally dL/dOPD) of a real loss L, writes
 *   grad_opd      device float[height][width] or NULL: dL/dOPD added to the
 *                 chain's own; absorbing: float[2][height][width], dL/dOPD then
 *                 dL/dtau
 *   grad_soa      device float[OSOG_D][ld] (absorbing: [OSOG_D_ABS][ld]) or NULL:
 *                 dL/d(cx, cy, angle, a, b, height, dn[, dmu]); row OSOG_SHAPE
 *                 is written as 0
 *   grad_globals  device float[4] or NULL: dL/d(defocus, shear, bias), [3] = 0
 * Forward intermediates are recomputed inside the call, not stored.  Shot
 * noise is treated as a constant.  workspace: >= osog_workspace_size(...,
 * with_backward = 1) bytes. */
osog_status osog_render_backward(osog_context* ctx, void* stream, int32_t height, int32_t width,
                                 const float* soa, int64_t n, int64_t ld,
                                 const osog_optics* optics, const float* globals,
                                 const float* grad_intensity, const float* grad_opd,
                                 float* grad_soa, float* grad_globals,
                                 void* workspace, size_t workspace_bytes);

/* One frame of a batch (host array of these; pointers are device memory). */
typedef struct {
  int32_t height, width;
  const float* soa;
  int64_t n, ld;
  osog_optics optics;
  const float* globals;      /* device float[4]                               */
  float* opd_out;            /* device float[height][width] or NULL           */
  float* intensity_out;      /* device float[height][width]                   */
} osog_frame;

/* Bytes of device workspace for osog_batch_render over these frames. */
osog_status osog_batch_workspace_size(osog_context* ctx, const osog_frame* frames,
                                      int32_t n_frames, int32_t pairs_per_particle,
                                      size_t* bytes);

/* Render many frames of uneven size and particle count in one launch of a HIP
 * graph, captured once per batch signature (frame descriptors, workspace,
 * timestamp buffer, per-size tiling and FFT radix, branch count) and replayed
 * on later calls with the same signature.  The graph holds one kernel chain per
 * frame (the launches osog_render makes) on `group` concurrent branches (see
 * osog_set_batch_group); every dependency is a graph edge.  Each frame's output
 * is bitwise identical to osog_render of that frame with the same tiling.
 * Asynchronous on `stream`.
 *   frame_done_ns  device uint64[n_frames + 1] or NULL: GPU timestamp (ns, the
 *                  device's constant-rate clock) at which each frame finished,
 *                  and [n_frames] = the batch start, for latency percentiles. */
osog_status osog_batch_render(osog_context* ctx, void* stream, const osog_frame* frames,
                              int32_t n_frames, void* workspace, size_t workspace_bytes,
                              uint64_t* frame_done_ns);

/* Number of frames of the last batch on this workspace in which some tile was
 * rasterised by the slower id-ordered scan of all particles (a segment of more
 * than 512 ids, or one past the pair list's capacity; the result is the same),
 * into *flag (host).  Waits for the device. */
osog_status osog_batch_error(osog_context* ctx, void* workspace, int32_t* flag);

/* Batch scheduling: the number of concurrent branches of the batch graph,
 * frame f on branch f mod group (0: the maximum, 8).  Default 4. */
osog_status osog_set_batch_group(osog_context* ctx, int32_t group);

/* Tiling used for frames of one canvas size in batches (the autotuner's
 * choice); other sizes use osog_set_tiling's. */
osog_status osog_set_size_tiling(osog_context* ctx, int32_t height, int32_t width, int32_t tile_h,
                                 int32_t tile_w);

/* FFT plan for frames of one canvas size: the largest Stockham radix, 8
 * (default) or 4.  Renders of that size in osog_render, osog_render_backward
 * and osog_batch_render use it. */
osog_status osog_set_size_radix(osog_context* ctx, int32_t height, int32_t width, int32_t fft_radix);

/* Autotuner: renders this frame `reps` times for every candidate plan -- tile
 * shape 16x16, 8x32 or 32x8 and FFT radix 8 or 4 -- timed with HIP events on
 * the stream (waits for the device), and records the fastest for frames of
 * this canvas size (as osog_set_size_tiling / osog_set_size_radix would).
 * Writes the choice and its mean milliseconds per render.  workspace: as for
 * osog_render. */
osog_status osog_autotune(osog_context* ctx, void* stream, int32_t height, int32_t width, const float* soa,
                          int64_t n, int64_t ld, const osog_optics* optics, const float* globals,
                          float* intensity_out, void* workspace, size_t workspace_bytes, int32_t reps,
                          int32_t* tile_h, int32_t* tile_w, int32_t* fft_radix, float* best_ms);

/* Binning only (steps F1-F4 of the renderer), for inspection and testing:
 * writes the pairs sorted by (tile key, particle id):
 *   keys_out, pids_out  device int32[capacity]; pair_count_out device int32[1]
 *   tile_start_out      device int32[n_tiles + 1]; counts_out device int32[n] or NULL
 * n_tiles = (height / tile_h) * (width / tile_w).  *pair_count_out is the full
 * pair count; if it exceeds `capacity`, keys_out and pids_out are not written.
 * workspace: as for osog_render (its pair list is filled as a render fills it;
 * a tile the raster would scan is produced by the same id-ordered scan). */
osog_status osog_bin(osog_context* ctx, void* stream, int32_t height, int32_t width,
                     const float* soa, int64_t n, int64_t ld, int32_t* keys_out,
                     int32_t* pids_out, int64_t capacity, int32_t* pair_count_out,
                     int32_t* tile_start_out, int32_t* counts_out, void* workspace,
                     size_t workspace_bytes);

/* ---- Learned initializer (a BF16 CNN on the MFMA matrix cores) ----------------
 * Six 3x3 convolutions (padding 1, bias + ReLU, channels 1->32/2, 32->32,
 * 32->64/2, 64->64, 64->128/2, 128->128/2), global average pooling, dense
 * 128->64 (ReLU) and 64->4.  Input images enter as I / 4 - 1 (the empty DIC
 * background at bias pi/2 maps to 0); the four outputs are the caller's
 * normalised targets.
 * Parameters are one FP32 vector (layout: for each convolution W[3][3][Ci][Co]
 * then b[Co]; then W[128][64], b[64], W[64][4], b[4]); convolutions run in
 * BF16 with FP32 accumulation; training is deterministic. */
osog_status osog_cnn_param_count(int64_t* count);
/* Workspace for a batch of `batch` images of height x width (multiples of 16). */
osog_status osog_cnn_workspace_size(int32_t batch, int32_t height, int32_t width, size_t* bytes);
/* pred (device float[batch][4]) = network(images (device float[batch][height][width])). */
osog_status osog_cnn_forward(osog_context* ctx, void* stream, int32_t batch, int32_t height, int32_t width,
                             const float* images, const float* params, float* pred, void* workspace,
                             size_t workspace_bytes);
/* One training step on a batch: forward, mean squared error against targets
 * (device float[batch][4]) into *loss (device float[1], or NULL), backward
 * through every layer, and, when step >= 1, an Adam update (beta1 0.9, beta2
 * 0.999, eps 1e-8, bias correction for `step`) of params with moments m, v
 * (device float[count] each).  grads_out (device float[count] or NULL)
 * receives the gradient.  step = 0 computes the gradient only. */
osog_status osog_cnn_train_step(osog_context* ctx, void* stream, int32_t batch, int32_t height, int32_t width,
                                const float* images, const float* targets, float* params, float* m, float* v,
                                int32_t step, float lr, float* loss, float* grads_out, void* workspace,
                                size_t workspace_bytes);
/* One 3x3 convolution (padding 1, stride 1 or 2) on the MFMA kernels, NHWC BF16
 * (uint16 bit patterns):
 *   mode 0  out_bf16[B][Ho][Wo][Co] = relu(conv(x, w) + bias)
 *   mode 1  out_bf16[B][Hi][Wi][Ci] = dL/dx given grad_y and the layer output y (ReLU mask)
 *   mode 2  out_f32[3][3][Ci][Co]   = dL/dw given x, grad_y and y
 * w is [3][3][Ci][Co] BF16.  workspace: osog_conv3x3_workspace_size bytes. */
osog_status osog_conv3x3_workspace_size(int32_t mode, int32_t batch, int32_t height, int32_t width,
                                        int32_t c_in, int32_t c_out, int32_t stride, size_t* bytes);
osog_status osog_conv3x3(osog_context* ctx, void* stream, int32_t mode, int32_t batch, int32_t height,
                         int32_t width, int32_t c_in, int32_t c_out, int32_t stride, const uint16_t* x,
                         const uint16_t* y, const uint16_t* grad_y, const uint16_t* w, const float* bias,
                         uint16_t* out_bf16, float* out_f32, void* workspace, size_t workspace_bytes);

/* Polyhedral crystal habits (paper Eq. 1: a habit is the intersection of M
 * half-spaces) for particles whose table row OSOG_SHAPE holds 2 + k (habit k).
 * Habit k, in unit coordinates (U, V, W), is {n_x U + n_y V + n_z W <= d} over
 * its faces; a particle of it occupies (x, y) = c + R(angle) (a U, b V),
 * z = height W, and its thickness at a pixel is the length of the vertical ray
 * through the pixel centre inside the solid.  Micro-topography (the procedural
 * high-frequency perturbation of the height map): where that thickness is
 * positive it becomes max(0, t + amplitude r(x, y)), r value noise on a square
 * lattice of `cell` px in canvas coordinates, lattice values 2u - 1 from the first
 * word of the Philox4x32-10 block at counter (lattice x, lattice y, k, 3) under
 * topo_seed (u as for the shot noise), blended with smoothstep weights.
 *   face_counts   host int32[n_habits], 4..32 faces each
 *   faces         host float[sum counts][4]: (n_x, n_y, n_z, d), habit after habit
 *   radius        host float[n_habits]: a bound on sqrt(U^2 + V^2) over the habit
 *                 (it sets the particle's pixel box: max(a, b) radius + 1)
 *   topo_amplitude_um, topo_cell_px  host float[n_habits] (amplitude >= 0; cell a
 *                 power of two in [1, 256])
 * Each habit must be a bounded, non-empty polytope (checked by enumerating its
 * vertices) whose vertices lie within `radius`.  Replaces the context's habits
 * (n_habits = 0 clears them); a table row naming an undefined habit adds
 * nothing.  Synchronous (uploads a small table). */
osog_status osog_set_habits(osog_context* ctx, int32_t n_habits, const int32_t* face_counts, const float* faces,
                            const float* radius, const float* topo_amplitude_um, const float* topo_cell_px,
                            uint64_t topo_seed);

/* ---- Spectral loss of Eq. 8 (targets that cannot be aligned pixel by pixel) -----
 * With F the unnormalised 2-D DFT and eps > 0 inside the logarithms,
 *   A(k) = log(|F(image)(k)| + eps) - log(|F(target)(k)| + eps),
 *   L = (1/(H W)) sum over the H x W bins of A(k)^2,
 *   dL/dimage = Re(DFT(g)), g(k) = (2/(H W)) A(k) conj(F(k)) / (|F(k)| (|F(k)| + eps)).
 * The loss sees amplitudes only: a circular shift of the image leaves it
 * unchanged.  height, width: powers of two in [32, 4096].  Asynchronous on
 * `stream`; workspace: osog_spectral_workspace_size bytes (device). */
osog_status osog_spectral_workspace_size(int32_t height, int32_t width, size_t* bytes);
/* target_logamp (device float[height * width], written): log(|F(target)| + eps)
 * in the library's spectrum layout (bin (ky, kx) at kx * height + ky, kx and ky
 * in DFT order), computed once per target. */
osog_status osog_spectral_target(osog_context* ctx, void* stream, int32_t height, int32_t width,
                                 const float* target, float eps, float* target_logamp, void* workspace,
                                 size_t workspace_bytes);
/* loss_out (device float[1]): L of image (device float[height][width]) against a
 * target_logamp from osog_spectral_target with the same eps; grad_out (device
 * float[height][width] or NULL): dL/dimage. */
osog_status osog_spectral_loss(osog_context* ctx, void* stream, int32_t height, int32_t width,
                               const float* image, const float* target_logamp, float eps, float* loss_out,
                               float* grad_out, void* workspace, size_t workspace_bytes);

/* The in-band spectrum columns the chain carries for these optics: signed kx in
 * [*kx_lo, *kx_lo + *kx_n) are the columns with at least one DFT bin inside the
 * (oblique: shifted) pupil disc (Eq. 3).  Host only, no device work. */
osog_status osog_band_info(const osog_context* ctx, int32_t height, int32_t width,
                           const osog_optics* optics, int32_t* kx_lo, int32_t* kx_n);

/* The counter-based generator of the shot noise, Philox4x32-10 (Salmon et al.,
 * SC'11), evaluated on the device: out[4k..4k+3] = philox(ctr[4k..4k+3], key). */
osog_status osog_philox4x32_10(void* stream, const uint32_t* ctr, int64_t count, uint32_t key0,
                               uint32_t key1, uint32_t* out);

/* Per-stage timing with HIP events.  While enabled, every call records a pair
 * of events around each stage on the caller's stream (this adds a little
 * launch overhead).  osog_profile_read waits for the recorded events, adds
 * their elapsed milliseconds into ms[OSOG_NSTAGES] and the number of timed
 * launches into launches[OSOG_NSTAGES] (both host arrays, overwritten), and
 * forgets them. */
enum {
  OSOG_STAGE_BINNING = 0,   /* F1-F4: boxes and counts, scan (tile offsets), emit */
  OSOG_STAGE_RASTER = 1,    /* F5: per-tile OPD accumulation                      */
  OSOG_STAGE_PASS1 = 2,     /* F6: exp(i phi), row FFT, band store                */
  OSOG_STAGE_PASS2 = 3,     /* F7: column FFT, transfer function, column IFFT     */
  OSOG_STAGE_PASS3 = 4,     /* F8: row IFFT, |E|^2, shot noise                    */
  OSOG_STAGE_ADJ_PASS3 = 5,
  OSOG_STAGE_ADJ_PASS2 = 6,
  OSOG_STAGE_ADJ_PASS1 = 7,
  OSOG_STAGE_ADJ_RASTER = 8,
  OSOG_STAGE_BATCH = 9,     /* a whole batch graph launch                          */
  OSOG_NSTAGES = 10
};
osog_status osog_profile_enable(osog_context* ctx, int32_t enable);
osog_status osog_profile_read(osog_context* ctx, double* ms, int64_t* launches);

const char* osog_status_string(osog_status s);
const char* osog_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* OSOG_H */

/*
 * rsim.h - C ABI of librsim: MI355X (gfx950) FMCW radar echo synthesis.
 *
 * The problem, as stated in Section 3 of "A Simulation Method for MMW Radar Sensing
 * in Traffic Intersection Based on BART Algorithm" (arXiv 2208.10939): vehicles with
 * positions and velocities in an intersection (Section 3.1, Table 1), a radar
 * transmitting FMCW chirps (eq. (8)) from P Tx to Q Rx antennas, whose echo
 * (eqs. (7), (9)-(13)) is sampled into an O x M x N cube (O = P Q channels, M samples
 * per chirp, N chirps) and turned into a range-Doppler map by FFTs over samples and
 * chirps (Section 3.3).
 *
 * Conventions
 *  - Every call returns an int32 status: RSIM_OK (0) or a negative RSIM_E* code. On
 *    failure rsim_last_error() describes it; outputs are then undefined.
 *  - The caller owns every buffer it passes. Host inputs are copied before the call
 *    returns. Device outputs are written asynchronously on the given HIP stream
 *    (hipStream_t passed as void*, NULL = default stream) and are valid only once
 *    that stream has completed the work.
 *  - A context is not thread-safe: one context per host thread.
 *  - World frame of the paper (Table 1): Z up, Y along the lanes, metres, seconds, Hz.
 *  - Complex values are interleaved (re, im). Echo layout H[scene][o][n][m] with
 *    channel o = p * Q + q.
 */
#ifndef RSIM_H
#define RSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSIM_ABI_VERSION 2

/* status codes */
#define RSIM_OK 0
#define RSIM_EINVAL (-1)  /* bad argument: NULL, NaN/Inf, index out of range, bad id  */
#define RSIM_ENOMEM (-2)  /* device allocation failed or exceeded rsim_set_mem_limit  */
#define RSIM_EDEVICE (-3) /* HIP error, no device, or a device call on a host-only ctx */
#define RSIM_ESTATE (-4)  /* waveform, array or scene missing / inconsistent          */
#define RSIM_ERANGE (-5)  /* supported-size limit exceeded (see each call)             */

/* precision of rsim_synthesize / rsim_form_rdm */
#define RSIM_FP32_PHASE64 0 /* FP64 geometry and phase reduction, FP32 sum; complex64 */
#define RSIM_FP64 1         /* FP64 throughout; complex128 echo                       */

/* facet-sum kernel of rsim_synthesize (FP32 sum) */
#define RSIM_KERNEL_AUTO 0   /* the fastest eligible kernel for this array and waveform as    */
                             /* timed by rsim_autotune; the vector units until it has run      */
#define RSIM_KERNEL_VECTOR 1 /* vector units: full phase factorisation incl. the cross term   */
#define RSIM_KERNEL_MATRIX 2 /* matrix cores: separable Tx x Rx contraction per sample, which  */
                             /* drops the Tx-Rx cross term; eligible when |2 pi slope d_p e_q| */
                             /* <= 1e-5 rad, P <= 12 and Q <= 16                               */
#define RSIM_KERNEL_NUFFT 3  /* type-1 non-uniform FFT over the sample index: each facet's    */
                             /* divided-difference integral spread onto a 2x-oversampled grid  */
                             /* per channel with a Taylor-expanded Gaussian, then an FFT and   */
                             /* deconvolution (relative error ~1e-5 or below). Exact per-      */
                             /* channel distances (no cross-term approximation). Eligible for  */
                             /* n_g = the smallest 2^a 3^b >= 2M in 32..2048 and every channel  */
                             /* within 2.5 grid cells of the phase-centre path (aperture, and  */
                             /* with intra_chirp twice the largest Doppler shift of a source,  */
                             /* n_g (f0 + M df) 2 v_max / (c fs) cells). Ground bounce and     */
                             /* intra_chirp are supported (the latter to first order in the    */
                             /* sample time and in its m^2 phase term). Facets                 */
                             /* spanning more than 1.5 grid cells (2 r_max df n_g / c, r_max   */
                             /* the largest vertex-to-centroid distance of the scenes' meshes) */
                             /* are split into 4, 16 or 64 midpoint sub-triangles; beyond 12   */
                             /* cells the kernel is ineligible.                                */

/* visibility-mask mode */
#define RSIM_MASK_COMPUTE 0 /* compute the lit-facet mask; write it to vis_mask if given */
#define RSIM_MASK_INPUT 1   /* use vis_mask (device) as given; skip the visibility step */

typedef struct rsim_ctx rsim_ctx;

/* FMCW waveform (eq. (8), Section 4.1). Sample m of chirp n is taken at frequency
 * f_m = f0 + m * slope / fs and chirp start time t_n = n * chirp_period.
 * n_samples (M) and n_chirps (N) in 1..4096; the RDM calls need lengths 2^a 3^b. */
typedef struct {
  double f0_hz;
  double slope_hz_per_s;
  double fs_hz;
  double chirp_period_s;
  int32_t n_samples;
  int32_t n_chirps;
} rsim_waveform;

/* Options of rsim_synthesize / rsim_form_rdm. Zero-initialised = defaults. */
typedef struct {
  int32_t precision; /* RSIM_FP32_PHASE64 (default) or RSIM_FP64                         */
  int32_t mask_mode; /* RSIM_MASK_COMPUTE (default) or RSIM_MASK_INPUT                   */
  int32_t use_graph; /* batched call: capture the launches in a hipGraph and replay it  */
  int32_t persistent;/* batched call: one persistent facet-sum launch over a work queue  */
  int32_t timing;    /* record per-stage HIP events (read with rsim_last_timings)        */
  int32_t tile_m;    /* facet-sum samples per thread (0 = autotuned/default)              */
  int32_t tile_f;    /* facets staged per LDS tile (0 = default). Compiled (tile_m,      */
                     /* tile_f): FP32 16x16 32x8 32x16 64x8 64x16, FP64 8x8 16x8; others  */
                     /* fail with RSIM_EINVAL                                            */
  int32_t intra_chirp; /* 0: stop-and-hop, geometry and delay frozen at t_n (default).   */
                     /* 1: the propagation delay of eq. (12) taken at each sample time  */
                     /* t_n + m / fs (range-Doppler coupling within a chirp); amplitude, */
                     /* facet integral and lit set stay at t_n. FP32 sum only.          */
  int32_t kernel;    /* RSIM_KERNEL_AUTO (default), _VECTOR, _MATRIX or _NUFFT; MATRIX or   */
                     /* NUFFT where ineligible fails with ERANGE (with RSIM_FP64: EINVAL);  */
                     /* AUTO falls back to VECTOR there                                     */
  int32_t census;    /* NUFFT facet sum: also count its records by source form (read with */
                     /* rsim_last_census); no effect on the results. Not with use_graph    */
  int32_t reserved[2];
} rsim_opts;

/* ---- context ---------------------------------------------------------------------- */

int32_t rsim_abi_version(void);

/* Create a context on HIP device `hip_device`. hip_device = -1 creates a host-only
 * context: meshes, scenes, waveform and array can be set and validated (and the BVH
 * built) but every device call returns RSIM_EDEVICE. On failure *out is NULL and
 * rsim_last_error(NULL) holds the message. */
int32_t rsim_create(int32_t hip_device, rsim_ctx **out);
void rsim_destroy(rsim_ctx *ctx);

/* Message of the last failing call on ctx (ctx = NULL: last failure of this thread
 * outside any context). Valid until the next call on the same ctx / thread. */
const char *rsim_last_error(const rsim_ctx *ctx);

/* Cap on the library's device allocations in bytes (0 = no cap). A call that would
 * exceed it fails with RSIM_ENOMEM. */
int32_t rsim_set_mem_limit(rsim_ctx *ctx, uint64_t bytes);

/* ---- scene ------------------------------------------------------------------------ */

/* Triangle mesh in its body frame: verts_xyz [n_verts][3] float32 metres, tris
 * [n_tris][3] int32 vertex indices, counter-clockwise = outward normal. The data are
 * copied and a bounding-volume hierarchy is built once here. Zero-area triangles are
 * accepted: they never scatter and never block. EINVAL on NaN/Inf or bad indices;
 * ERANGE beyond 2^26 triangles. */
int32_t rsim_load_mesh(rsim_ctx *ctx, const float *verts_xyz, int64_t n_verts,
                       const int32_t *tris, int64_t n_tris, int32_t *mesh_id);

int32_t rsim_create_scene(rsim_ctx *ctx, int32_t *scene_id);

/* Rigid instance of a mesh moving at constant velocity (eq. (12), Section 3.2):
 * world position x(t) = rot * x_body + pos0 + vel * t. rot is row-major 3x3 and
 * must be orthonormal. The scene's facets are numbered instance by instance in the
 * order instances were added. At most 4096 instances per scene. */
int32_t rsim_add_instance(rsim_ctx *ctx, int32_t scene_id, int32_t mesh_id,
                          const double rot[9], const double pos0[3], const double vel[3],
                          int32_t *inst_id);

/* Point scatterers (the point target of eq. (13)): pos0 [n][3], vel [n][3] float64,
 * amp_re_im [n][2] float64 complex amplitude s in m^2 (echo term s/(4 pi R_t R_r)). */
int32_t rsim_add_points(rsim_ctx *ctx, int32_t scene_id, const double *pos0,
                        const double *vel, const double *amp_re_im, int64_t n);

/* Replace a mesh's body-frame vertices (same count; triangles unchanged), e.g. for a
 * gradient step or a finite-difference probe. The BVH is rebuilt. Synchronous: waits
 * for queued work on the device first. */
int32_t rsim_update_mesh(rsim_ctx *ctx, int32_t mesh_id, const float *verts_xyz,
                         int64_t n_verts);

/* Replace an instance's start position and velocity (eq. (12)). Synchronous. */
int32_t rsim_set_instance_motion(rsim_ctx *ctx, int32_t scene_id, int32_t inst_id,
                                 const double pos0[3], const double vel[3]);

/* Number of facets F of a scene (sum over its instances) and words per chirp of its
 * lit-facet mask, ceil(F / 32). */
int32_t rsim_scene_info(rsim_ctx *ctx, int32_t scene_id, int64_t *n_facets,
                        int64_t *mask_words_per_chirp);

/* ---- radar ------------------------------------------------------------------------ */

int32_t rsim_set_waveform(rsim_ctx *ctx, const rsim_waveform *wf);

/* Antenna element positions in the world frame (Section 2.1, Fig. 3): tx [n_tx][3],
 * rx [n_rx][3] float64. 1..64 elements each. The Tx and Rx phase centres are the
 * element means; they define visibility and the facet-integral directions. */
int32_t rsim_set_array(rsim_ctx *ctx, const double *tx_xyz, int32_t n_tx,
                       const double *rx_xyz, int32_t n_rx);

/* Ground double bounce (Section 2.2: forward and backward rays joined after
 * reflections). enable = 1 adds the paths that reflect once on the flat road plane
 * z = z_ground on the transmit side, on the receive side, or on both, by the image
 * method: each is the single-bounce facet term with mirrored elements, times gamma
 * (complex reflection coefficient; -1 for a perfectly conducting plane) per bounce.
 * A facet takes a reflected side when its centroid lies above the plane, it faces the
 * mirrored phase centre, and both legs (centroid -> specular point -> phase centre) are
 * clear; instances lying in the plane (the road surface) do not block those legs.
 * While enabled, rsim_synthesize's vis_mask holds 4 mask sets per scene (path types
 * 0: direct, 1: Tx side reflected, 2: Rx side reflected, 3: both; type-major), the
 * persistent form is refused (EINVAL) and rsim_backward differentiates all four path types
 * (gamma held fixed).
 * ERANGE if an array element does not lie above the plane. Point scatterers take all
 * four paths. */
int32_t rsim_set_ground(rsim_ctx *ctx, int32_t enable, double z_ground, double gamma_re,
                        double gamma_im);

/* Facet-to-facet double bounce (Section 2.2: a ray followed as the facets reflect it and
 * a ray from the other end joined on a facet). With enable = 1, rsim_synthesize adds for
 * each chirp the paths T -> A -> B -> R over pairs of facets, each found from both ends:
 * a ray launched from a phase centre E (the Tx one, then the Rx one) reflects specularly
 * off the centroid of facet A (lit from E: facing it, unblocked) and first hits facet B,
 * which must face the image E' of E in A's plane and the other phase centre O with the
 * segment hit point -> O clear. The connection's echo is gamma / 2 times the facet term of
 * eqs. (7), (9)-(13) of the footprint of A's reflected tube on B's plane (the central
 * projection from E' of A's vertices, taken whole, not clipped to B) with E's elements
 * replaced by their images in A's plane; the two launching ends of a path each give half.
 * Connections are kept when every projection parameter exceeds 1/2 and the footprint lies
 * within 1.5 times the scene's largest facet radius of its centroid. Point scatterers
 * take no double bounce. gamma: complex reflection coefficient (-1: perfect conductor).
 * Runs in the NUFFT facet sum only: rsim_synthesize then fails with EINVAL for
 * RSIM_KERNEL_VECTOR / MATRIX, RSIM_FP64, intra_chirp, persistent or the ground plane,
 * with ERANGE where the NUFFT is ineligible (its window also holds the footprints); the
 * lit mask covers the single-bounce path only. A caller's vis_mask buffer then holds,
 * after each scene's N * mask_words words, that scene's connection table [2][N][F]
 * int32: for the ray launched from the Tx (first plane) or Rx (second) end at chirp n and
 * facet A, the facet B it connects to, or -1 (output with RSIM_MASK_COMPUTE, input with
 * RSIM_MASK_INPUT; a given entry outside 0 .. F-1 means no connection). rsim_backward
 * differentiates the connections with the table held (the NUFFT adjoint only: see there);
 * rsim_autotune fails with ESTATE while it is on. EINVAL for enable not 0/1 or a
 * non-finite gamma.
 * Device memory: 16 N F + 8 N bytes per scene for the connections. */
int32_t rsim_set_double_bounce(rsim_ctx *ctx, int32_t enable, double gamma_re, double gamma_im);

/* ---- echo and RDM ------------------------------------------------------------------ */

/* Echo frequency response H (Sections 2.2, 3.2; eqs. (7), (9)-(13)) of each scene:
 *   H[o,n,m] = sum over lit facets f of  j o_f I_f(k_m) / (4 pi R_t R_r)
 *              * exp(-j 2 pi (f_m tau - slope tau^2 / 2)),  tau = (R_t + R_r) / c,
 * with I_f the closed-form physical-optics integral over the triangle, o_f the
 * obliquity, R_t / R_r the distances from the facet centroid to Tx element p and
 * Rx element q, geometry frozen at t_n (stop-and-hop); plus point scatterers.
 * The beat signal of eq. (13) is conj(H).
 *   echo     DEVICE, [n_scenes][O][N][M] complex64 (complex128 with RSIM_FP64).
 *   vis_mask DEVICE or NULL, [sum over scenes of N * mask_words(scene)] uint32,
 *            bit f%32 of word [n][f/32] = facet f lit at chirp n; output with
 *            RSIM_MASK_COMPUTE, input with RSIM_MASK_INPUT (then required).
 * ESTATE without waveform/array; EINVAL for an unknown scene id; ERANGE if the
 * array aperture is too large for the phase factorisation (see DESIGN notes in
 * rsim_set_array's error message). */
int32_t rsim_synthesize(rsim_ctx *ctx, const int32_t *scene_ids, int32_t n_scenes,
                        void *echo, uint32_t *vis_mask, void *hip_stream,
                        const rsim_opts *opts);

/* Range-Doppler processing (Section 3.3; eqs. (4), (5), (10)-(11)) of n_cubes echo
 * cubes [O][N][M]: beat x = conj(H), X = FFT over m, Y = FFT over n with zero Doppler
 * moved to row N/2, rdm = |Y|^2. Unnormalised FFTs, no window.
 *   echo  DEVICE [n_cubes][O][N][M] complex64 (complex128 with RSIM_FP64)
 *   rdm   DEVICE [n_cubes][O][N][M] float32 (float64 with RSIM_FP64), row = Doppler
 *   y_opt DEVICE or NULL, Y in the echo's complex type and layout.
 * ERANGE unless M and N are of the form 2^a 3^b in 2..4096 (mixed radix-2/3 FFT). */
int32_t rsim_form_rdm(rsim_ctx *ctx, const void *echo, int32_t n_cubes, void *rdm,
                      void *y_opt, void *hip_stream, const rsim_opts *opts);

/* rsim_form_rdm for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. Same arguments, layouts,
 * outputs and errors as rsim_form_rdm; it calls no hipMalloc, hipFree or allocating
 * routine. Its work memory (twiddle tables, then the range-transformed planes of up to
 * g = floor((32 MiB - twiddles) / (N M csize)) channel planes at a time, csize 8 or 16
 * bytes) is one file-scope device array of 32 MiB per GPU, held from library load until
 * the process ends and shared by every call on that GPU: calls that overlap on one GPU
 * (other streams, threads or contexts) race. ERANGE when one N x M plane and its
 * twiddles do not fit the 32 MiB (e.g. N = M = 2048 at FP32). opts->timing records
 * the whole call as stage 3. */
int32_t rsim_form_rdm_noalloc(rsim_ctx *ctx, const void *echo, int32_t n_cubes, void *rdm,
                              void *y_opt, void *hip_stream, const rsim_opts *opts);

/* Per-stage device times (ms) of the last rsim_synthesize / rsim_form_rdm /
 * rsim_backward call made with opts.timing = 1, measured with HIP events on the
 * caller's stream. Blocks until those events complete. Stage order:
 * 0 visibility, 1 compaction, 2 facet sum (incl. FP64 prep), 3 range FFT,
 * 4 Doppler FFT + RDM, 5 adjoint facet sum, 6 adjoint FFTs, 7 vertex gather,
 * 8 the NUFFT spread kernel alone (summed over its launches; part of stage 2),
 * 9 the NUFFT adjoint's gather kernels alone (part of stage 5).
 * Stages not run report 0. n_stages up to 10. */
int32_t rsim_last_timings(rsim_ctx *ctx, float *ms, int32_t n_stages);

/* Record census of the last rsim_synthesize call that ran the NUFFT facet sum with
 * opts.census set: counts[k] = (lit facet or point, chirp) records whose grid sources take
 * form k: 0 none (zero-area facet), 1 three point Gaussians (one per vertex: the divided
 * difference of the facet integral when every pair of vertex phases differs by more than
 * 2 rad), 2 a point Gaussian and a quadratic-weighted one (one close pair), 3 one
 * quadratic-weighted Gaussian about the centroid (a small facet, or a point scatterer).
 * The spread's work per (record, channel) follows from them. Blocks until that call's
 * work is done. ESTATE if no such call ran on ctx. */
int32_t rsim_last_census(rsim_ctx *ctx, int64_t counts[4]);

/* ---- adjoint ------------------------------------------------------------------------ */

/* Gradient of a real loss L through the echo of one scene (FP32 path), with the
 * lit-facet mask held fixed and chirps recomputed rather than stored (stop-and-hop
 * geometry, or the delay within the chirp after rsim_set_backward_intra_chirp(ctx, 1);
 * with the ground plane on, all four path types).
 * With the facet-to-facet double bounce on, the connections too, their table held: each
 * connection's adjoint sums (its footprint's node offsets and amplitude, and the distance
 * from every channel element, the launching side's mirrored in A's plane) are carried
 * through the footprint construction to the vertices of A and B, whose derivatives are
 * taken by FP64 central differences (step 1e-6 m); those gradients are added with FP64
 * atomics, so their last bits depend on arrival order. That runs in the NUFFT adjoint,
 * stop-and-hop, without the ground plane and for at most 32 Tx + Rx elements: EINVAL with
 * the ground plane, rsim_set_backward_intra_chirp(ctx, 1) or a backward kernel of
 * RSIM_KERNEL_VECTOR / MATRIX; ERANGE where the NUFFT adjoint is ineligible or for more
 * elements. Device memory: 144 F bytes and, per chirp of a chunk, 2 F (32 + 4 (P + Q))
 * bytes beside the NUFFT adjoint's work, whose record lists grow to 3 F entries.
 *   grad_echo  DEVICE [O][N][M] complex64: dL/dRe(H) + j dL/dIm(H)
 *   vis_mask   DEVICE mask of that scene from the forward call (N * mask_words; four
 *              sets with the ground plane; with the double bounce followed by the
 *              connection table [2][N][F] int32 of that call)
 *   grad_verts host array of n_meshes DEVICE pointers, each [n_verts][3] float32 of
 *              the scene's meshes in mesh-id order (NULL entries skipped); dL/dx_body
 *              summed over the instances of each mesh, ACCUMULATED into the buffers.
 *   grad_vel   DEVICE [n_instances][3] float64, dL/dvel per instance, overwritten.
 */
int32_t rsim_backward(rsim_ctx *ctx, int32_t scene_id, const void *grad_echo,
                      const uint32_t *vis_mask, float *const *grad_verts, int32_t n_meshes,
                      double *grad_vel, void *hip_stream);

/* Facet-sum kernel of rsim_backward (Sections 2.2, 3.2; eqs. (7), (9)-(13), differentiated):
 * RSIM_KERNEL_AUTO (default) takes the NUFFT adjoint where it is eligible for the scene
 * (grid of at most 2048 cells; node offsets 2 r_max df n_g / c plus the array's channel
 * offsets below half the grid, r_max the largest vertex-to-centroid distance), else the
 * matrix cores when the array
 * allows them (the same eligibility as rsim_opts.kernel: |2 pi slope d_p e_q| <= 1e-5 rad,
 * P <= 12, Q <= 16), else the vector units; RSIM_KERNEL_VECTOR always the vector units;
 * RSIM_KERNEL_MATRIX the matrix cores and RSIM_KERNEL_NUFFT the NUFFT adjoint (a type-2
 * transform: the echo gradient through the transposed FFT and deconvolution onto each
 * channel's grid, then Gaussian-weighted moments gathered per lit facet), rsim_backward then
 * failing with ERANGE where ineligible. EINVAL for another value. All give the same
 * gradients to FP32 rounding, the dropped cross term and the NUFFT's error (relative
 * <= 1e-5); all three are deterministic (a fixed order of operations, no atomics) except
 * for the double bounce's connections (rsim_backward). */
int32_t rsim_set_backward_kernel(rsim_ctx *ctx, int32_t kernel);

/* Which forward rsim_backward differentiates (Section 3.2, eq. (12) at the sample times):
 * enable = 0 (default) the stop-and-hop echo; 1 the echo synthesized with
 * rsim_opts.intra_chirp = 1 (each facet's delay taken at t_n + m / fs, its centroid moving
 * with its velocity within the chirp; amplitude, facet integral and lit set at t_n). The
 * velocity gradient then gains the sum over samples of (m / fs) times the phase's
 * derivative in the centroid. That adjoint runs on the vector units: with enable = 1,
 * RSIM_KERNEL_AUTO takes them and rsim_backward fails with EINVAL for a backward kernel of
 * RSIM_KERNEL_MATRIX or RSIM_KERNEL_NUFFT. The phase's derivatives take the delays and unit
 * vectors at t_n (they move by v m / fs within a chirp: relative changes near 1e-6).
 * EINVAL for enable not 0/1. Device memory while enabled: 16 N F slots + 12 N F bytes
 * (slots = sample tiles x channel tiles of the vector-unit adjoint). */
int32_t rsim_set_backward_intra_chirp(rsim_ctx *ctx, int32_t enable);

/* Work buffers of the NUFFT facet sum and its adjoint (RSIM_KERNEL_NUFFT): per chirp the
 * grid cells, sorted positions and records of every possible entry (facets, points, and
 * with the double bounce two connections per facet), the runs and their windows of O x 32
 * grid cells (forward), or O grids of n_g cells (adjoint). A call runs its chirps in chunks
 * that fit 48 GiB, half the device memory free at the call and the context's memory limit;
 * max_chirps > 0 caps the chunk further (less device memory, more launches), 0 restores
 * the default. Results do not depend on the chunking (the same bits). EINVAL for
 * max_chirps < 0. Takes effect at the next call (a captured graph is re-captured). */
int32_t rsim_set_nufft_chunk(rsim_ctx *ctx, int32_t max_chirps);

/* Gradient of L with respect to the echo given dL/dP of the power RDM P = |Y|^2 and
 * the Y of the forward call (FP32): dL/dY = 2 (dL/dP) Y, then the adjoint of the
 * Doppler and range transforms (Section 3.3).
 *   grad_rdm DEVICE [n_cubes][O][N][M] float32, y DEVICE complex64 same layout,
 *   grad_echo DEVICE complex64 [n_cubes][O][N][M]: dL/dRe(H) + j dL/dIm(H). */
int32_t rsim_rdm_backward(rsim_ctx *ctx, const float *grad_rdm, const void *y, int32_t n_cubes,
                          void *grad_echo, void *hip_stream);

/* Gradient of L with respect to the echo given dL/dRe(Y) + j dL/dIm(Y) of the
 * Doppler-FFT output (adjoint of rsim_form_rdm's linear part, FP32):
 *   grad_y DEVICE [n_cubes][O][N][M] complex64 -> grad_echo same layout. */
int32_t rsim_rdm_adjoint(rsim_ctx *ctx, const void *grad_y, int32_t n_cubes,
                         void *grad_echo, void *hip_stream);

/* ---- detection, point cloud, noise ------------------------------------------------- */

/* CA-CFAR and angle-FFT settings (Section 3.3; the paper leaves window sizes and the
 * threshold open, so they are parameters). Around each cell under test: guard cells
 * on each side (Doppler rows, range bins), then training cells on each side beyond
 * them; noise = mean power over the training ring, both axes periodic. A cell is
 * detected when its power exceeds scale x noise. The angle FFT runs over the virtual
 * array on its half-wavelength grid, zero-padded to na_x x na_z. */
typedef struct {
  int32_t guard_doppler, guard_range;
  int32_t train_doppler, train_range;
  float scale;       /* threshold factor on the training mean, > 0                      */
  int32_t na_x;      /* angle FFT length along x, 2^a 3^b; 0 = smallest >= 2 x extent    */
  int32_t na_z;      /* along z; 0 = as na_x (1 when the virtual array is one row)       */
  int32_t max_points;/* points written per cube, >= 1                                    */
} rsim_cfar_opts;

/* One detected range-Doppler cell and its point. */
typedef struct {
  int32_t row, bin;           /* Doppler row (zero Doppler at row N/2) and range bin     */
  float power, noise;         /* channel-integrated power and the CFAR noise estimate   */
  float range_m;              /* eq. (4): bin x c / (2 B)                                */
  float velocity_mps;         /* eq. (5): (row - N/2) x lambda_c / (2 N T_c), + receding */
  float u, w;                 /* direction cosines along x and z from the angle peak     */
  float x, y, z;              /* point: phase-centre midpoint + range (u, sqrt(1-u^2-w^2), w) */
  float angle_power;          /* |angle spectrum|^2 at the peak                          */
  int32_t kx, kz;             /* signed angle bins of the peak                           */
  int32_t reserved[2];
} rsim_point;

/* Detection and point cloud of n_cubes RDM frames (Section 3.3; eq. (6)): the channel-
 * integrated map P[n][m] = sum_o rdm[o][n][m], CA-CFAR on P, then for each detected
 * cell (row-major order) the 2-D angle FFT of Y over the virtual-array grid, whose
 * first maximum gives u = -2 kx / na_x, w = -2 kz / na_z (Y comes from the beat signal
 * conj(H), so a target in direction d carries phases exp(-j k d . v) across the
 * virtual elements v = tx_p + rx_q).
 *   rdm        DEVICE [n_cubes][O][N][M] float32 (rsim_form_rdm, FP32)
 *   y          DEVICE [n_cubes][O][N][M] complex64 (rsim_form_rdm's y_opt)
 *   det_mask   DEVICE [n_cubes][N][M] uint8 or NULL: 1 = detected
 *   noise_map  DEVICE [n_cubes][N][M] float32 or NULL: CFAR noise estimate
 *   points     DEVICE [n_cubes][max_points] rsim_point: the first max_points detections
 *   n_points   DEVICE [n_cubes] int32: number of detections (may exceed max_points)
 * EINVAL for bad settings; ERANGE when the window does not fit the map (2 (guard +
 * train) + 1 > N or M), when the virtual elements are not on a half-wavelength grid
 * in one x-z plane, or when an angle length is not 2^a 3^b or exceeds the LDS. */
int32_t rsim_detect(rsim_ctx *ctx, const float *rdm, const void *y, int32_t n_cubes,
                    const rsim_cfar_opts *opts, uint8_t *det_mask, float *noise_map,
                    rsim_point *points, int32_t *n_points, void *hip_stream);

/* Adds complex white Gaussian noise at snr_db to n_cubes echo cubes in place (Section
 * 3.2): sigma^2 = mean |H|^2 of the cube / 10^(snr_db / 10), each part variance
 * sigma^2 / 2. Normals from Philox4x32-10 (counter = element index lo, hi, cube, 0;
 * key = seed lo, hi) through Box-Muller in FP64, so a given seed gives the same noise
 * on any device.
 *   echo DEVICE [n_cubes][O][N][M] complex64 (complex128 with opts->precision =
 *   RSIM_FP64); opts may be NULL. */
int32_t rsim_add_noise(rsim_ctx *ctx, void *echo, int32_t n_cubes, double snr_db,
                       uint64_t seed, void *hip_stream, const rsim_opts *opts);

/* ---- tuning ------------------------------------------------------------------------- */

/* Time the facet-sum tile shapes (and the matrix-core and NUFFT kernels where eligible)
 * on the given scenes and keep the fastest as the
 * default for this (M, O, precision); optionally append it to a JSON-lines cache
 * file (cache_json_path may be NULL). Synchronous. */
int32_t rsim_autotune(rsim_ctx *ctx, const int32_t *scene_ids, int32_t n_scenes,
                      const char *cache_json_path);

/* Wait for all work the library queued on hip_stream. */
int32_t rsim_sync(rsim_ctx *ctx, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* RSIM_H */

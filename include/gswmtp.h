/*
 * gswmtp.h - C ABI of the MI355X (gfx950) GSW-MTP hologram library.
 *
 * The library computes phase-only holograms (CGHs) for arbitrary optical focus
 * arrays with the weighted Gerchberg-Saxton iteration of Liu et al.,
 * "Fast generation of arbitrary optical focus array" (arXiv:2206.12661),
 * Algorithm 1, in which the diffraction step is the matrix triple product of
 * Eq. 2,  Theta = Omega_y E Omega_x,  Omega_x = exp(-i 2 pi K_x^T X),
 * Omega_y = exp(-i 2 pi Y^T K_y),  evaluated only at the foci, with all-zero
 * pupil rows/columns and non-focus focal samples removed (Sec. 2, Fig. 1).
 *
 * Conventions used by every call:
 *   - The pupil is ny x nx samples, row-major (row j <-> y / v_j, column i <->
 *     x / u_i).  Phase arrays are float32 [ny*nx]; complex arrays are float32
 *     interleaved (re, im).
 *   - The kernel phase of a pupil sample (u, v) and a focus (x, y) is
 *     -2 pi (s_x u x + s_y v y)  (sign of Eq. 1).  With u, v in pixels and
 *     s_x = 1/nx, s_y = 1/ny, focal coordinates are in units of lambda f/(N du).
 *   - Foci keep the caller's order in every per-focus array.
 *   - Every call returns an int status: GSWMTP_OK (0) or a negative
 *     GSWMTP_E_* code; gswmtp_last_error() gives a message for the last
 *     failing call on a plan.  No C++ exception crosses this boundary.
 *   - A plan is not thread-safe; distinct plans are independent.
 *   - Streams: every plan orders its GPU work after work already queued on the
 *     caller's stream (the one given at creation or by gswmtp_set_stream; NULL
 *     is the default stream) and makes that stream wait for it, so device
 *     pointers passed to *_device calls may be produced and consumed on the
 *     caller's stream without extra synchronisation.  Calls with host output
 *     buffers return after the data is copied.
 *   - Ownership: gswmtp_plan_create deep-copies every input array; the caller
 *     may free or modify them afterwards.  Output buffers belong to the
 *     caller.  The library frees only what it allocated.
 */
#ifndef GSWMTP_H
#define GSWMTP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSWMTP_VERSION 100

/* Status codes. */
enum {
    GSWMTP_OK = 0,
    GSWMTP_E_INVAL = -1,          /* bad size, pointer, non-finite or negative input */
    GSWMTP_E_DUPFOCUS = -2,       /* two foci with identical (x, y, z) */
    GSWMTP_E_EMPTYAPERTURE = -3,  /* amplitude (after mask) is zero everywhere */
    GSWMTP_E_NOMEM = -4,          /* host or device allocation failed, or workspace too small */
    GSWMTP_E_HIP = -5,            /* a HIP runtime call failed */
    GSWMTP_E_NONFINITE = -6,      /* a focus intensity sum became non-finite */
    GSWMTP_E_NODEV = -7,          /* no usable gfx950 device */
    GSWMTP_E_UNSUPPORTED = -8     /* valid request the library does not implement */
};

/* Arithmetic of the two dense complex products (forward and adjoint MTP).
 *   FP32:   float32 operands, float32 MFMA (v_mfma_f32_32x32x2_f32).
 *   BF16X3: each operand split x = hi + lo in bfloat16; products
 *           hi*hi + hi*lo + lo*hi on bf16 MFMA with float32 accumulation.
 *   FP16X3: the same with float16 halves (operands pre-scaled by powers of 2).
 *   BF16X6: three-term bfloat16 split, six products.
 * Kernel-matrix phases are always reduced in float64; focus statistics are
 * always reduced in float64. */
typedef enum {
    GSWMTP_FP32 = 0,
    GSWMTP_BF16X3 = 1,
    GSWMTP_FP16X3 = 2,
    GSWMTP_BF16X6 = 3
} gswmtp_precision;

/* Focal-field update rule (Algorithm 1, weight update).
 *   GSW:  generalised weighting w <- w sqrt(t / i) (the paper's method).
 *   GS:   no weighting (w stays 1): the plain Gerchberg-Saxton baseline. */
typedef enum {
    GSWMTP_WEIGHT_GSW = 0,
    GSWMTP_WEIGHT_GS = 1
} gswmtp_weighting;

/* Plan descriptor.  Fill with gswmtp_desc_init, then set fields.
 * All pointers are HOST pointers and are copied by gswmtp_plan_create. */
typedef struct gswmtp_desc {
    int ny, nx;                   /* pupil samples, 1..16384 each */
    const float *amplitude;       /* [ny*nx] >= 0, finite; NULL = all ones.
                                     Zero marks samples outside the aperture. */
    const uint8_t *mask;          /* [ny*nx]; NULL = all ones.  Effective
                                     amplitude is mask ? amplitude : 0. */
    const double *u;              /* [nx] pupil x coordinates; NULL = i-(nx-1)/2 */
    const double *v;              /* [ny] pupil y coordinates; NULL = j-(ny-1)/2 */
    double s_x, s_y;              /* kernel phase scales, finite and non-zero */
    int n_foci;                   /* 1..262144 */
    const double *fx, *fy;        /* [n_foci] focus coordinates, finite */
    const double *target;         /* [n_foci] target intensities, >= 0, sum > 0 */
    const float *phi0;            /* [ny*nx] initial phase, finite; NULL = zeros */
    int precision;                /* gswmtp_precision */
    int axis;                     /* -1 auto, 0 reduce along y, 1 along x */
    int weighting;                /* gswmtp_weighting */
    const double *fz;             /* [n_foci] axial focus positions, finite;
                                     NULL = all foci on the focal plane.  A
                                     focus at z multiplies its kernel rows and
                                     columns by the pupil's defocus phase
                                     exp(i pi z (s u)^2) along x and
                                     exp(i pi z (s v)^2) along y (the 3-D
                                     extension of Eq. 2 through the lens's
                                     quadratic phase; separable per axis), so
                                     the reduced grid holds (coordinate, z)
                                     pairs per axis. */
} gswmtp_desc;

/* Index information of a plan (the reduced focal grid and pupil compaction). */
typedef struct gswmtp_index_info {
    int n_foci;
    int ux, uy;                   /* unique focus (x, z) / (y, z) pairs
                                     (unique x / y when every z is 0) */
    int ny_kept, nx_kept;         /* pupil rows / columns with any non-zero amplitude */
    int axis;                     /* 0: dense product over the y foci (M = uy); 1: over x */
    int n_aperture;               /* samples with amplitude > 0 */
    double sum_a2;                /* sum of amplitude^2 over the pupil */
} gswmtp_index_info;

typedef struct gswmtp_plan gswmtp_plan;
typedef struct gswmtp_batch gswmtp_batch;

/* Library version (GSWMTP_VERSION of the build). */
int gswmtp_version(void);

/* Human-readable name of a status code (static string, never NULL). */
const char *gswmtp_status_string(int status);

/* Message of the last failed call on plan p (static "" if none); with
 * p == NULL, the message of the calling thread's last failed plan creation. */
const char *gswmtp_last_error(const gswmtp_plan *p);

/* Fill d with defaults: all pointers NULL, s_x = s_y = 0 (must be set),
 * precision FP32, axis -1, weighting GSW.  Returns GSWMTP_E_INVAL if d == NULL. */
int gswmtp_desc_init(gswmtp_desc *d);

/* Build a plan on the current HIP device (Algorithm 1 inputs: A, phi0,
 * target intensities, w0 = 1, focus coordinates).
 * Validates every input on the host first (GSWMTP_E_INVAL, no GPU use), then
 * runs the plan kernels: effective amplitude and compaction, unique focal
 * coordinates and gather indices (GSWMTP_E_DUPFOCUS on a repeated (x, y, z);
 * -0.0 and +0.0 are one coordinate), axis choice (fewer unique coordinates,
 * ties to y), kernel matrices (phase reduced in float64), E0 = A exp(i phi0).
 * Synchronises once to size the product buffers.  stream: hipStream_t or NULL.
 * On failure *out is NULL and nothing is leaked; gswmtp_last_error(NULL)
 * holds the message.
 * Testing the failure paths: with the environment variable
 * GSWMTP_FAULT_INJECT=alloc (read at each call) every device allocation of
 * the call fails - it returns GSWMTP_E_NOMEM after validating d, before any
 * device work; with GSWMTP_FAULT_INJECT=alloc:K only the K-th allocation
 * fails (the plan makes two: index pool, product pool), and what was built
 * is released.  The same applies to gswmtp_batch_create (its allocations:
 * the tuner's scratch, then its pool); gswmtp_plan_create_with_workspace
 * allocates nothing and ignores it. */
int gswmtp_plan_create(gswmtp_plan **out, const gswmtp_desc *d, void *stream);

/* Device memory a plan for d needs (both of its pools), in bytes, computed on
 * the host from the descriptor alone (no GPU work, no allocation): the same
 * index counts and layout the plan derives (unique focal coordinates, kept
 * pupil rows and columns, axis, padded product sizes, tile schedules for the
 * current device's CU count, or 256 without one).  The environment switches
 * that change the layout must be the same at plan creation.  GSWMTP_E_INVAL
 * or GSWMTP_E_EMPTYAPERTURE as gswmtp_plan_create would return them. */
int gswmtp_plan_workspace_size(const gswmtp_desc *d, size_t *bytes);

/* gswmtp_plan_create with the plan's device memory carved from dev_ws, a
 * DEVICE buffer of `bytes` bytes (at least gswmtp_plan_workspace_size),
 * 256-byte aligned, owned by the caller and left untouched by the library
 * except as the plan's storage; it must stay valid until
 * gswmtp_plan_destroy, which does not free it (e.g. a torch tensor from the
 * caching allocator).  The plan makes no device allocation of its own
 * besides what HIP's stream, event and graph objects hold.
 * GSWMTP_E_INVAL for a null, empty or misaligned buffer; GSWMTP_E_NOMEM,
 * with the size needed in gswmtp_last_error(NULL), when it is too small. */
int gswmtp_plan_create_with_workspace(gswmtp_plan **out, const gswmtp_desc *d, void *dev_ws,
                                      size_t bytes, void *stream);

/* Free a plan (NULL-safe).  Waits for its queued work first. */
int gswmtp_plan_destroy(gswmtp_plan *p);

/* Change the caller stream used for ordering (NULL = default stream). */
int gswmtp_set_stream(gswmtp_plan *p, void *stream);

/* Block until all work queued by p has finished. */
int gswmtp_sync(gswmtp_plan *p);

/* Queue n_iter >= 0 passes of Algorithm 1 (forward MTP, foci intensities,
 * accuracy xi, termination test, weight update, focal-field update, adjoint
 * MTP, phase-only projection).  If stop_accuracy > 0, a pass whose forward
 * field has xi > stop_accuracy ends the run before updating anything; later
 * queued passes do nothing.  Asynchronous: returns once the work is queued.
 * Passes are replayed from a captured HIP graph unless the environment
 * variable GSWMTP_NO_GRAPH is set to a non-zero value. */
int gswmtp_iterate(gswmtp_plan *p, int n_iter, double stop_accuracy);

/* Camera in the loop (the experiments of Sec. 2): queue ONE pass of
 * Algorithm 1 whose weight update takes the focus intensities from
 * measured [n_foci] (host, caller order; finite, >= 0, positive sum) -
 * intensities captured for the CURRENT phase - in place of the computed
 * |Theta|^2; they are normalised to unit sum on the device like the computed
 * ones.  Everything else is an ordinary pass: the new focal field keeps
 * arg Theta of the computed forward field (or the frozen phases under phase
 * fixing), the history records the computed field's statistics, the pass
 * is counted, no termination test is taken.  With GS weighting the
 * intensities have no effect.  The caller decides when to switch (the paper
 * switches once the computed accuracy xi reaches 0.95).  Synchronises
 * before returning, so measured may be reused at once.  Runs eagerly (not
 * from the captured graph of gswmtp_iterate). */
int gswmtp_iterate_measured(gswmtp_plan *p, const double *measured);

/* Total passes that updated the phase since creation or the last set_state
 * (synchronises). */
int gswmtp_iterations_done(gswmtp_plan *p, int *n);

/* Current phase phi - the hologram Algorithm 1 outputs, the argument of the
 * pupil field after the phase-only projection of its last pass - in
 * (-pi, pi], 0 outside the aperture: host [ny*nx], row-major.  Synchronises. */
int gswmtp_get_phase(gswmtp_plan *p, float *out);
/* Same into device memory [ny*nx] (stream-ordered, no host sync). */
int gswmtp_get_phase_device(gswmtp_plan *p, float *dev_out);

/* Replace the current phase (host / device [ny*nx], finite, row-major): the
 * pupil field becomes E = A exp(i phi), the input of Algorithm 1's forward
 * step.  Weights and the iteration count are kept.  GSWMTP_E_INVAL for a
 * non-finite host phase (the device form is not scanned). */
int gswmtp_set_phase(gswmtp_plan *p, const float *phi);
int gswmtp_set_phase_device(gswmtp_plan *p, const float *dev_phi);

/* Focal field Theta of the CURRENT phase at every focus (caller order): the
 * forward matrix triple product of Eq. 2 evaluated at the foci, as in the
 * first step of each pass of Algorithm 1.  Interleaved complex [2*n_foci]
 * (re, im) on the host.  Runs the forward product when the phase changed
 * since the last one.  Synchronises. */
int gswmtp_get_foci_field(gswmtp_plan *p, float *out);
/* Same into device memory, stream-ordered, no host sync: dev_field [2*n_foci]
 * receives Theta, dev_intensity [n_foci] the intensities I = |Theta|^2 of
 * Algorithm 1; either may be NULL, not both (GSWMTP_E_INVAL). */
int gswmtp_get_foci_field_device(gswmtp_plan *p, float *dev_field, float *dev_intensity);

/* Statistics of the CURRENT phase's focal field (any output pointer may be
 * NULL):
 *   xi  - the intensity accuracy of Algorithm 1, 1 - ||t - i|| / ||i|| with
 *         i = I / sum I and t = Itilde / sum Itilde (normalised, so the scale
 *         of the targets does not matter);
 *   eta - the diffraction efficiency of the Fig. 2 caption, energy at the
 *         foci over the incident energy: sum I / (N_ap sum A^2), N_ap the
 *         pupil samples with A > 0.  The foci's samples of the focal plane
 *         are not orthogonal (foci closer than the diffraction limit share
 *         energy), so eta can exceed 1 for such patterns;
 *   uniformity - 1 - (max r - min r) / (max r + min r), r = i / t over the
 *         foci with t > 0 (1 when every focus meets its target).
 * Runs the forward product when the phase changed.  Synchronises. */
int gswmtp_get_stats(gswmtp_plan *p, double *xi, double *eta, double *uniformity);

/* The weighting factors w of Algorithm 1 (the generalised weighting of
 * Sec. 2; all ones at plan creation), [n_foci] float64 on the host, caller
 * order.  set_weights replaces them (finite, else GSWMTP_E_INVAL); both
 * synchronise. */
int gswmtp_get_weights(gswmtp_plan *p, double *out);
int gswmtp_set_weights(gswmtp_plan *p, const double *w);

/* Per-pass history of (xi, eta, uniformity) - as gswmtp_get_stats defines
 * them - of the field each pass of Algorithm 1 started from (the accuracy
 * the pass tested for termination), oldest first.  Copies min(cap, stored) entries (3 doubles each) of the
 * most recent passes; *n receives the number copied.  The ring keeps the last
 * 4096 passes. */
int gswmtp_get_history(gswmtp_plan *p, double *buf, int cap, int *n);

/* Checkpoint: phase [ny*nx], weights [n_foci], pass count.  set_state restores
 * all three and clears the history.  Either array may be NULL to skip it. */
int gswmtp_get_state(gswmtp_plan *p, float *phi, double *w, int *iters);
int gswmtp_set_state(gswmtp_plan *p, const float *phi, const double *w, int iters);

/* Phase fixing (the variant of Sec. 2 after Kim et al.): from the
 * from_pass-th updating pass on (counted like gswmtp_iterations_done, from 1),
 * the new focal field keeps the focal phases recorded by the first pass that
 * applies the rule, instead of arg Theta of each pass; the weights keep
 * updating.  from_pass = 0 turns it off.  Setting it (and set_phase /
 * set_state) clears the recorded phases.  Stream-ordered; GSWMTP_E_INVAL for
 * from_pass < 0. */
int gswmtp_set_phase_fixing(gswmtp_plan *p, int from_pass);

/* Index results (host).  info is required; each array may be NULL:
 * ix, iy [n_foci] gather indices; xu [ux], yu [uy] sorted unique
 * coordinates; rows [ny_kept], cols [nx_kept] kept pupil rows/columns. */
int gswmtp_get_index(gswmtp_plan *p, gswmtp_index_info *info, int32_t *ix, int32_t *iy,
                     double *xu, double *yu, int32_t *rows, int32_t *cols);

/* Operator-level calls (do not touch the plan's phase, weights or history).
 * forward_field: Theta = P(E), the forward matrix triple product of Eq. 2,
 *   at the foci for an arbitrary complex pupil field E (host, interleaved
 *   [2*ny*nx], row-major); samples outside the kept rows/columns are ignored.
 *   Output host [2*n_foci], caller order.
 * adjoint_field: E' = P^H(Theta), the operator Algorithm 1 uses as its
 *   inverse, taken as the adjoint of Eq. 2 (the conjugate kernels, opposite
 *   exponent sign, no 1/N scale - the phase-only projection that follows in
 *   a pass discards any positive scale), for focal values Theta (host
 *   [2*n_foci]) with every other sample of the reduced focal grid zero;
 *   no projection.  Output host [2*ny*nx], zero outside the kept
 *   rows/columns.  Both synchronise; GSWMTP_E_INVAL for non-finite input. */
int gswmtp_forward_field(gswmtp_plan *p, const float *E, float *theta);
int gswmtp_adjoint_field(gswmtp_plan *p, const float *theta, float *E);

/* gswmtp_forward_field for callers that cannot allocate device memory (serving
 * loops and harnesses that forbid it): the same arguments, kernels and result,
 * bit for bit, but the call's scratch (staging of E, the compacted pupil or
 * its split planes, the grid form's intermediate products, the gather and
 * split-K partials, the output staging) lives in one static device array of
 * 64 MiB that the library holds on each GPU it runs on until the process
 * ends, instead of the plan's own buffers.  The call allocates nothing and
 * leaves the plan's buffers untouched.  Every call on a GPU shares that GPU's
 * array (it keeps the last call's contents; the call clears it first), so
 * calls that overlap on one GPU - from several host threads, on any plans -
 * race; calls from one thread are ordered, since each returns after its
 * result is copied out.  GSWMTP_E_NOMEM, with the bytes needed in
 * gswmtp_last_error(p), when the plan's sizes need more than 64 MiB
 * (roughly beyond 2.9 M pupil samples in FP32); GSWMTP_E_HIP if the array
 * cannot be located on the device. */
int gswmtp_forward_field_noalloc(gswmtp_plan *p, const float *E, float *theta);

/* Gradient of L = sum_n g_n |Theta_n|^2 with respect to the current phase:
 *   dL/dphi = 2 Im(conj(E) * P^H(g * Theta)),
 * with Theta the field of the current phase.  dev_g: device float [n_foci];
 * dev_grad: device float [ny*nx] (0 outside the aperture).  Stream-ordered. */
int gswmtp_phase_gradient_device(gswmtp_plan *p, const float *dev_g, float *dev_grad);
/* That gradient applied at once by one Adam step (the update of
 * gswmtp_adam_step_device, same arguments and errors) to the user-layout
 * phases phi and moments m, v (device float [ny*nx], in place), with the step
 * number t read from dev_step: the Adam kernel reads the gradient where the
 * adjoint product left it, so no gradient array is written or read.  The
 * same values as the two calls in a row, bit for bit.  Stream-ordered. */
int gswmtp_phase_gradient_adam_device(gswmtp_plan *p, const float *dev_g, float *phi, float *m,
                                      float *v, const float *dev_step, double lr, double beta1,
                                      double beta2, double eps);

/* The design loss of the differentiable form and its gradient in the
 * intensities, for the n foci intensities dev_I and targets dev_target (device
 * float [n], targets >= 0 with a positive sum):
 *   L = sum_n (i_n - t_n)^2 - eta_weight * eta,  i = I / sum I,
 *   t = T / sum T,  eta = sum I / (n_ap sum_a2)
 * (normalised intensities against normalised targets as in the weight update
 * of Algorithm 1; eta the diffraction efficiency of the Fig. 2 caption with the
 * incident energy of the discrete sums n_ap sum A^2), and
 *   dL/dI_k = 2 r_k / S - 2 sum_m r_m i_m / S - eta_weight / (n_ap sum_a2),
 * r = i - t, S = sum I.  dev_loss [1] and dev_dI [n] (device float) receive
 * them.  One workgroup, sums in float64 over a fixed order; stream-ordered on
 * `stream`, no host synchronisation.  GSWMTP_E_INVAL for n < 1, a null
 * pointer, or n_ap, sum_a2 not positive and finite. */
int gswmtp_design_loss_device(const float *dev_I, const float *dev_target, int n, double n_ap,
                              double sum_a2, double eta_weight, float *dev_loss, float *dev_dI,
                              void *stream);

/* gswmtp_design_loss_device plus the design loop's bookkeeping on the device,
 * so that a loop step needs no kernels besides the library's: after forming L,
 * with s = *dev_step (device float, the number of steps recorded so far),
 * dev_hist[s] = L when s < hist_cap, then *dev_step = s + 1 - the step number
 * t of the gswmtp_adam_step_device call that follows on the same stream.
 * dev_hist (device float [hist_cap]) may be NULL when hist_cap is 0.  Same
 * errors as gswmtp_design_loss_device, and GSWMTP_E_INVAL for a null dev_step
 * or hist_cap < 0. */
int gswmtp_design_loss_record_device(const float *dev_I, const float *dev_target, int n,
                                     double n_ap, double sum_a2, double eta_weight,
                                     float *dev_loss, float *dev_dI, float *dev_hist,
                                     int hist_cap, float *dev_step, void *stream);

/* One Adam step (Kingma and Ba's update with bias-corrected moments, the
 * optimiser of the differentiable form's design loop; not from the paper) on
 * n float32 values, all device memory, stream-ordered on `stream`
 * (hipStream_t, NULL = default), no host synchronisation and no allocation,
 * so a design step can be captured in a graph:
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   phi -= (lr / (1 - b1^t)) m / (sqrt(v) / sqrt(1 - b2^t) + eps),
 * with t read from dev_step (device float, the number of this step, >= 1;
 * the caller advances it before each call).  phi, m, v [n] are updated in
 * place; dev_grad [n] is read.  GSWMTP_E_INVAL for a null pointer (n > 0),
 * betas outside [0, 1), non-finite lr or eps < 0; n = 0 does nothing. */
int gswmtp_adam_step_device(float *phi, const float *dev_grad, float *m, float *v,
                            const float *dev_step, size_t n, double lr, double beta1,
                            double beta2, double eps, void *stream);

/* Profiling: run n_iter passes eagerly with HIP events around each stage on
 * the plan's stream and return the mean milliseconds per launch of each stage
 * in ms_out[GSWMTP_N_STAGES] (order: forward product with the fused focus
 * gather, focus update, scatter, adjoint product with the projection, and the
 * adjoint's split-K tail launch (0 work when the schedule has no tail: the
 * figure is then the event overhead alone)).  In the split precisions, when
 * every reduced row holds one focus, the scatter stage is the scaling of
 * Omega^H by the new focal values (the adjoint of Eq. 2 bracketed the other
 * way; no S is formed).  Changes the plan state exactly as
 * gswmtp_iterate(p, n_iter, 0) would. */
#define GSWMTP_N_STAGES 5
int gswmtp_time_stages(gswmtp_plan *p, int n_iter, double *ms_out);

/* Kernel names of the stages, for matching profiler output (static strings,
 * "" for a stage without a launch). */
const char *gswmtp_stage_kernel(gswmtp_plan *p, int stage);

/* Batched form: several independent plans (one hologram each, any sizes)
 * iterated together (an addition of this library; the paper computes one
 * hologram at a time).  Each pass runs Algorithm 1 on every plan: forward
 * product of Eq. 2 with the focus gather, weight update, scatter, adjoint
 * product with the phase-only projection.
 *
 * Products: every plan's forward and adjoint product falls in a shape class,
 * (product, padded M, N, K).  Each class has its own kernel configuration
 * (tile, loop, K chunks of the forward), chosen by an autotuner at
 * batch_create: every candidate valid for the shape is timed on the class's
 * own tiles, repeated until they fill the device twice, with the adjoint's
 * output sent to scratch (no plan state changes); the fastest wins.  Choices
 * are kept per process and, when the environment variable GSWMTP_TUNE_CACHE
 * names a file, in that JSON file (read at batch_create, rewritten when new
 * classes were tuned), keyed by architecture, CU count, precision, product
 * and (M, N, K).  GSWMTP_BATCH_TILE=BMxBN fixes the tile of every class it
 * divides; GSWMTP_BATCH_TILE=plan or GSWMTP_BATCH_NO_TUNE=1 gives each class
 * its plans' single-plan configuration (no K split).  A tuned class whose
 * timing of its product's dominant configuration is within 10% of its best
 * takes the dominant one.  The tiles of all plans go to one device work list
 * per configuration, longest K first, one launch each: a stage with one
 * configuration runs it persistently (the tiles dealt to the resident
 * workgroups on the host, longest first, each to the least-loaded one;
 * GSWMTP_BATCH_PERSIST=0: one workgroup per tile); a stage's several
 * configurations (at most 5) run as parallel branches of the captured graph
 * with one workgroup per tile.  Focus update and scatter are one grouped
 * launch each.
 *
 * batch_create: plans[n_plans] (1..65536 distinct plans on one device, all
 *   of one precision, else GSWMTP_E_INVAL) must outlive the batch; the
 *   batch keeps pointers, copies nothing.  Allocates its own work lists and
 *   argument tables (and tuning scratch while it tunes).  stream:
 *   hipStream_t or NULL.  GSWMTP_E_INVAL when the tuning cache cannot be
 *   written; GSWMTP_E_UNSUPPORTED when a stage would need more than five
 *   configurations.
 * batch_iterate: n_iter passes on every plan, each plan stopping on its own
 *   as gswmtp_iterate(p, n_iter, stop_accuracy) would; ordered after the
 *   caller's stream and each plan's queued work, and before later calls on
 *   the plans and the caller's stream.  Each plan's results equal those of
 *   gswmtp_iterate on that plan alone with no K split (GSWMTP_NO_SPLITK=1)
 *   bit for bit when its classes' configurations are the plan's own (as
 *   under GSWMTP_BATCH_TILE=plan), and to float32 rounding otherwise.  Read
 *   results through the plans.
 * batch_set_stream: the caller stream later batch_iterate calls are ordered with.
 * batch_sync: wait for the batch's queued passes.
 * batch_tiles: tiles[4] = forward BM, BN, adjoint BM, BN of the class with
 *   the most work of each product; tune_ms (nullable) [8] = that class's
 *   timed ms for the plain 64x64, 64x128, 128x64, 128x128 candidates
 *   (forward then adjoint; 0 = not timed).
 * batch_n_classes / batch_class_info: the shape classes and their
 *   configurations, with the tuning table of each (the candidates timed and
 *   their ms per copy of the class's tiles).
 * batch_tune_ms: host milliseconds batch_create spent timing candidates.
 * batch_last_error: message of the batch's last failed call, or of the last
 *   failed batch_create on this thread when b == NULL. */
#define GSWMTP_BATCH_MAX_CANDIDATES 8
typedef struct gswmtp_batch_class {
    int product;                  /* 0 forward (with the focus gather), 1 adjoint */
    int m, n, k;                  /* padded product sizes */
    int n_plans;                  /* plans in the class */
    int config[6];                /* BM, BN, BK, k-groups, loop (0 plain, 1 pipelined,
                                     2 direct, 3 16x16 blocks), forward K chunks */
    double ms;                    /* timed ms per copy of the class's tiles (0: not timed) */
    int source;                   /* 0 the plans' own or the only candidate, 1 tuned now,
                                     2 tuning cache, 3 GSWMTP_BATCH_TILE */
    int n_tried;
    int tried_config[GSWMTP_BATCH_MAX_CANDIDATES][6];
    double tried_ms[GSWMTP_BATCH_MAX_CANDIDATES];
} gswmtp_batch_class;
int gswmtp_batch_create(gswmtp_batch **out, gswmtp_plan *const *plans, int n_plans, void *stream);
int gswmtp_batch_iterate(gswmtp_batch *b, int n_iter, double stop_accuracy);
int gswmtp_batch_set_stream(gswmtp_batch *b, void *stream);
int gswmtp_batch_sync(gswmtp_batch *b);
int gswmtp_batch_tiles(const gswmtp_batch *b, int *tiles, double *tune_ms);
int gswmtp_batch_n_classes(const gswmtp_batch *b, int *n);
int gswmtp_batch_class_info(const gswmtp_batch *b, int i, gswmtp_batch_class *out);
int gswmtp_batch_tune_ms(const gswmtp_batch *b, double *ms);
const char *gswmtp_batch_last_error(const gswmtp_batch *b);
int gswmtp_batch_destroy(gswmtp_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* GSWMTP_H */

/*
 * liboct: MI355X (gfx950) library for model-based iterative reconstruction
 * (MBIR) of spectral-domain OCT with the ISAM system model
 * (Mason et al., "Model-based iterative reconstruction for spectral-domain
 * optical coherence tomography", Sec. 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Problem statement (Sec. 2.1, eq. (1)): image x in C^N, measurements
 * y in R^M.  N = batch * n_y * n_x * n_depth, M = batch * n_y * n_x * n_k
 * (n_y = 1 for a B-scan).
 *
 * Layouts (all buffers are device pointers, dense, A-scan contiguous):
 *   image        complex64 (interleaved float re, im), [batch][n_y][n_x][n_depth]
 *   measurement  float32,                                [batch][n_y][n_x][n_k]
 * Measurements are full length; pixels with mask 0 are ignored (eq. (7)).
 *
 * Arithmetic: complex FP32 with FP32 accumulation in the transforms; FP64
 * for the wavenumber-grid coordinates, the per-wavenumber phase tables, the
 * reductions (residual norm, objective, power-iteration norms) and the
 * FISTA momentum scalars.
 *
 * Ownership: the caller owns every data buffer; a plan owns its tables and
 * workspace (allocated by oct_plan_create, freed by oct_plan_destroy).
 * Execution: calls are asynchronous on the given stream (a hipStream_t passed
 * as void*, NULL = the default stream) unless stated otherwise.  One plan
 * must not be used from two streams at once.
 * Errors: no exception crosses the ABI.  Every call returns an oct_status;
 * oct_last_error() gives a message for the last failure of the calling thread.
 *   OCT_E_INVALID      null pointer, non-positive size, sigma * n_depth not an
 *                      integer, odd or unsupported kb_width, bad penalty
 *   OCT_E_UNSUPPORTED  a transform length with a prime factor above 7, sizes
 *                      beyond the kernels' limits, Haar with a dimension not
 *                      divisible by 2^levels
 *   OCT_E_NOMEM        device or host allocation failed
 *   OCT_E_DEVICE       a HIP runtime error
 */
#ifndef OCT_H
#define OCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oct_plan* oct_plan_t;

typedef enum {
  OCT_OK = 0,
  OCT_E_INVALID = 1,
  OCT_E_NOMEM = 2,
  OCT_E_DEVICE = 3,
  OCT_E_UNSUPPORTED = 4
} oct_status;

/* Regularisers R of Sec. 2.2: l1 with Psi = I (eq. (13)), isotropic total
 * variation (eq. (14)), and a multi-level orthonormal Haar wavelet l1. */
typedef enum { OCT_PEN_L1 = 0, OCT_PEN_TV = 1, OCT_PEN_HAAR = 2, OCT_PEN_DTCWT = 3 } oct_penalty;

/* Acquisition geometry (Sec. 2.1, eq. (4)-(9); optics of Sec. 3.1). */
typedef struct {
  int32_t lateral_dims;   /* 1 = B-scan (one lateral axis), 2 = volume          */
  int32_t kb_width;       /* J, Kaiser-Bessel taps: 4, 6 or 8                    */
  int64_t n_depth;        /* N_z image depth samples                             */
  int64_t n_x, n_y;       /* lateral A-scans (n_y = 1 for a B-scan)              */
  int64_t n_k;            /* M_k spectrometer pixels per A-scan (>= 2)           */
  int64_t batch;          /* independent problems of the same geometry           */
  double k_min, k_max;    /* rad/um; linear-k grid with inclusive endpoints      */
  double dx, dy;          /* lateral pitch, um                                   */
  double dz;              /* depth pitch, um; <= 0 selects pi / (2 N_z dk)       */
  double z_focus;         /* focal depth, um; < 0 selects floor(N_z/2) dz        */
  double beam_waist;      /* w0 (1/e^2 intensity radius), um; <= 0: no beam term */
  double disp_a, disp_b;  /* Omega_m = a (m-m_c)^2 + b (m-m_c)^3, m_c=(M_k-1)/2   */
  double oversamp;        /* sigma; K = sigma * N_z must be an integer            */
  double kb_beta;         /* KB shape; <= 0 selects pi sqrt(J^2/s^2 (s-1/2)^2-0.8)*/
  int32_t model;          /* oct_model: how K, Q and D of eq. (6)-(8) are formed  */
} oct_geometry;

/* The per-lateral-frequency part of Phi (eq. (5)-(8)).
 * OCT_MODEL_DIRECT: the NUFFT evaluated at beta_m(q) = sqrt(4 k_m^2 - q^2) of
 *   every spectrometer wavenumber, then the filter and e^{j Omega}; any n_k.
 * OCT_MODEL_LITERAL: the paper's chain as printed, for n_k = 2 n_depth: K
 *   samples the filtered spectrum at the N wavenumbers of the even pixels (the
 *   same NUFFT) and takes its N-point inverse DFT, Q pads to 2N, D is the
 *   2N-point DFT, then e^{j Omega}.  The odd pixels are the trigonometric
 *   interpolation D Q implies (equal to the direct model at q = 0).
 * Every entry point (forward, adjoint, gradient, solve, power iteration, the
 * paper's backward operator, the ISAM images) follows the plan's model; the
 * axial and dispersion-corrected images use the direct model at q = 0. */
typedef enum { OCT_MODEL_DIRECT = 0, OCT_MODEL_LITERAL = 1 } oct_model;

/* Create a plan: builds the FP64-derived tables (wavenumber grid, filter
 * phases, deapodisation, KB polynomial pieces, twiddles), packs the mask and
 * allocates the workspace on the current device.
 * mask: HOST pointer to uint8 [n_y][n_x][n_k] (nonzero = observed), shared by
 * the batch; NULL means every pixel is observed (Sec. 2.1, diag(s) of eq. (7)).
 * Synchronous. */
oct_status oct_plan_create(const oct_geometry* g, const uint8_t* mask, oct_plan_t* out);

/* Free a plan and everything it owns.  Synchronises the device first. */
oct_status oct_plan_destroy(oct_plan_t plan);

/* Free a plan without synchronising the device: for pools of plans (the
 * serving loop) that know the plan's work is complete, e.g. from an event
 * recorded after its last call; freeing a plan with work still pending on
 * some stream is undefined.  Plan memory comes from the device's
 * stream-ordered memory pool, whose freed blocks serve the next plans (the
 * library raises the pool's release threshold, so the process keeps them). */
oct_status oct_plan_release(oct_plan_t plan);

/* Upper bound of the device bytes a plan plus one oct_mbir_solve of the given
 * penalty hold (tables, workspace, solver state, and the lateral spectrum of
 * y that a solve on a fully observed plan keeps); used for admission control.
 * penalty < 0: the bound for a plan that runs every penalty and entry point
 * over its life (all solver states and optional buffers, which a plan keeps
 * once allocated).  Host-only, returns 0 for an invalid geometry. */
size_t oct_plan_footprint_bytes(const oct_geometry* g, int32_t penalty);

/* y = Phi x = diag(s) Re{ diag(e^{j Omega}) D Q K x }  (eq. (7)), computed as
 * lateral FFT, per-lateral-frequency KB-NUFFT at beta = sqrt(4k^2 - q^2)
 * (eq. (5)-(6)), beam/focus/dispersion filter, inverse lateral FFT, real part
 * and mask.  x: image (read), y: measurement (written). */
oct_status oct_forward(oct_plan_t plan, const void* x, float* y, void* stream);

/* x = Phi^H r, the exact adjoint of oct_forward under <a,b> = Re(a^H b)
 * (the operator used in the gradient of eq. (3)).  r: measurement (read,
 * masked on use), x: image (written). */
oct_status oct_adjoint(oct_plan_t plan, const float* r, void* x, void* stream);

/* x = Phi* r, the backward operator of eq. (10)-(11):
 * K^H D^H Q^T diag(e^{-j Omega}) A(s . r) with A(z) = Re z - j H(z), H the
 * Hilbert transform along the spectral axis of every A-scan, taken as the
 * discrete analytic signal (DFT over the n_k samples, negative frequencies
 * removed, positive ones below the Nyquist bin doubled, inverse DFT).  The
 * lateral and NUFFT parts are those of oct_adjoint.  Phi* is not the adjoint
 * of oct_forward: the two differ by the spectral-edge leakage of the
 * analytic signal.  r: measurement (read, masked on use), x: image (written).
 * OCT_E_UNSUPPORTED when n_k has a prime factor above 7. */
oct_status oct_adjoint_paper(oct_plan_t plan, const float* r, void* x, void* stream);

/* g = Phi^H (Phi x - y), the gradient of eq. (2)-(3).  half_resid_sq: device
 * double, receives 1/2 ||diag(s)(Phi x - y)||^2 summed over the batch;
 * may be NULL.  With every pixel observed (s = 1) the residual's lateral
 * round trip F_lat(Re F_lat^{-1} W - y) / N_lat equals W_h / N_lat -
 * F_lat(y) / N_lat, W_h the Hermitian part of W over q, and the norm is
 * taken by Parseval over the lateral frequencies: the same values up to
 * rounding, without the inverse and forward lateral passes (a volume's
 * oct_grad and every solve and power iteration take this route; a B-scan's
 * oct_grad keeps its one-pass seam, which costs less than forming F_lat(y)
 * per call). */
oct_status oct_grad(oct_plan_t plan, const void* x, const float* y, void* g,
                    double* half_resid_sq, void* stream);

/* z = prox_{lambda delta R}(v) over the constraint set C of eq. (16).
 * bound: C = {x : |x_i| <= bound} (a modulus bound per pixel, the complex
 * form of a box) when bound > 0 and finite; 0, negative or +inf: C = C^N;
 * NaN: OCT_E_INVALID.
 * OCT_PEN_L1: complex soft threshold by tau = lambda * delta, then the
 *   modulus clipped to the bound (exact: the constrained problem is radial).
 * OCT_PEN_TV with a bound: the constrained fast gradient projection (the
 *   primal point projected onto C in every step and at the end).
 * OCT_PEN_HAAR with a bound: OCT_E_UNSUPPORTED (no closed form).
 * OCT_PEN_TV: isotropic TV over the depth and lateral axes (forward
 *   differences, zero at the last index), solved by tv_inner steps of the fast
 *   gradient projection on the dual; state, if not NULL, is the dual
 *   (complex64 [lateral_dims + 1][image]) used as the warm start and
 *   overwritten with the new dual; NULL starts from zero.
 * OCT_PEN_HAAR: haar_levels-level orthonormal Haar over the depth and lateral
 *   axes, soft threshold on the detail bands.
 * OCT_PEN_DTCWT (Sec. 2.2): haar_levels-level dual-tree complex wavelet
 *   transform W over the depth and lateral axes (B-scan: four separable
 *   orthonormal trees scaled by 1/2, six oriented complex subbands per level;
 *   volume: eight trees scaled by 2^-3/2, 28 subbands; filters of the
 *   common-factor Hilbert-pair design, see oct_dtcwt_filter),
 *   z = W^T soft_tau(W v) with every complex detail coefficient's modulus
 *   shrunk by tau, low bands kept.  Dimensions divisible by 2^haar_levels
 *   (levels 1..5 for a B-scan, 1..4 for a volume); a bound gives
 *   OCT_E_UNSUPPORTED.
 * v and z are images and may not alias. */
oct_status oct_prox(oct_plan_t plan, int32_t penalty, double lambda, double delta,
                    int32_t tv_inner, int32_t haar_levels, double bound, const void* v, void* z,
                    void* state, void* stream);

/* Lowpass analysis filter of the DT-CWT (host, no device work): which = 0/1
 * first level of tree a/b, 2/3 later levels of tree a/b.  Writes up to 16
 * taps to h0 (host) and their count to *n; the highpass is
 * h1[k] = (-1)^k h0[n-1-k].  OCT_E_INVALID for another `which`. */
oct_status oct_dtcwt_filter(int32_t which, float* h0, int32_t* n);

/* Power iteration on Phi^H Phi (the Lipschitz constant behind the step size of
 * Sec. 2.3): x_0 = u / ||u|| with u from the SplitMix64 counter generator
 * (element e: real part u(2e), imaginary part u(2e+1), u uniform in [-1,1)
 * from the top 53 bits), then iters steps of x <- w / ||w||, w = Phi^H Phi x.
 * flags = OCT_SOLVE_PAPER_BACKWARD iterates Phi* Phi instead (Phi* of
 * oct_adjoint_paper; not self-adjoint, ||w|| then tends to its spectral
 * radius); 0 otherwise.  Writes the last ||w|| to *L_out (host).  A w of
 * zero norm stays zero (Phi = 0 on the plan's mask: nothing observed), so
 * *L_out is then exactly 0.  Synchronous. */
oct_status oct_lipschitz(oct_plan_t plan, int32_t iters, uint64_t seed, int32_t flags,
                         double* L_out, void* stream);

typedef enum {
  /* gradient step with the backward operator of eq. (10)-(11) (oct_adjoint_paper)
   * in place of the exact adjoint Phi^H */
  OCT_SOLVE_PAPER_BACKWARD = 1
} oct_solve_flags;

typedef struct {
  int32_t penalty;        /* oct_penalty                                          */
  int32_t iters;          /* FISTA iterations K (>= 1)                            */
  int32_t tv_inner;       /* inner FGP steps for TV (>= 1)                        */
  int32_t haar_levels;    /* Haar levels (>= 1)                                   */
  int32_t power_iters;    /* power-iteration steps when delta <= 0               */
  int32_t flags;          /* OR of oct_solve_flags (0: exact adjoint gradient)    */
  uint64_t seed;          /* power-iteration start vector seed                    */
  double lambda;          /* regularisation weight (absolute)                     */
  double delta;           /* step size; <= 0 selects 1 / (1.05 L_power), L_power
                             from oct_lipschitz with these flags (L_power = 0:
                             constant data term, every step admissible: 1)      */
  double bound;           /* modulus bound of the constraint set C of eq. (16)
                             (as in oct_prox; 0 = none)                           */
  const void* x0;         /* device image, start point; NULL = zero               */
  const double* lambda_item; /* HOST [batch] or NULL: a regularisation weight per
                             batch item (lambda is then unused); see below       */
  const void* z_prev0;    /* device image or NULL: z^{k0-1} of a resumed solve
                             (NULL: x0)                                            */
  void* z_prev_out;       /* device image or NULL: receives z^{K-1} (with x_out's
                             z^K, the state a later solve resumes from)            */
  int32_t k0;             /* iterations already done (>= 0): the momenta continue
                             from t_{k0+1}; k0 > 0 needs x0 = z^{k0}               */
} oct_solve_params;

/* Largest batch that oct_solve_params.lambda_item may describe. */
#define OCT_MAX_LAMBDA_ITEMS 64

typedef struct {
  double delta_used;      /* step size actually used                              */
  double lipschitz_est;   /* power-iteration estimate (0 when delta was given)    */
  double* objective;      /* HOST [iters] or NULL: 1/2||Phi x^k - y||^2 +
                             lambda R(z^k) per iteration                          */
} oct_solve_report;

/* FISTA (Sec. 2.3, eq. (15)): x^1 = x0, z^0 = x^1, t^1 = 1;
 * Resume: a solve of K iterations with x0 = z^k0, z_prev0 = z^{k0-1} and k0
 * continues a solve that has run k0 iterations; the two together equal one
 * solve of k0 + K iterations bitwise (for TV the dual warm start continues
 * from the plan's own last solve: resume on the plan that ran the first part,
 * with nothing else solved on it in between).
 * Per-item weights (lambda_item != NULL): item b solves its own problem with
 * weight lambda_item[b] > 0 (e.g. the candidates of the lambda search of
 * Sec. 3.2 on one measurement replicated over the batch).  Every penalty is
 * positively homogeneous, R(c x) = c R(x) for c > 0, so the FISTA iterates of
 * (y_b, lambda_b) are s_b times those of (y_b / s_b, lambda_0) with
 * s_b = lambda_b / lambda_0 (the gradient step and momentum are linear, and
 * prox_{tau R}(c v) = c prox_{(tau/c) R}(v)); the solve runs every item at
 * lambda_0 = max_b lambda_b on measurements scaled by 1 / s_b (a plan buffer
 * of n_meas floats, allocated on first use) and scales item b of z^K by s_b.
 * Requires batch <= OCT_MAX_LAMBDA_ITEMS, no bound, no objective report and no
 * x0 (OCT_E_UNSUPPORTED otherwise); OCT_E_INVALID for a weight <= 0 or NaN.
 * z^k = prox(x^k - delta Phi^H(Phi x^k - y)) (with OCT_SOLVE_PAPER_BACKWARD:
 * Phi*(Phi x^k - y), the operator of oct_adjoint_paper); t^{k+1} = (1 + sqrt(1 + 4 t_k^2))/2;
 * x^{k+1} = z^k + (t^k - 1)/t^{k+1} (z^k - z^{k-1}).  Writes z^K to x_out.
 * y: measurement (read), x_out: image (written).  Synchronous when a report
 * with an objective array or a power iteration is requested, otherwise
 * asynchronous. */
oct_status oct_mbir_solve(oct_plan_t plan, const float* y, const oct_solve_params* params,
                          void* x_out, oct_solve_report* report, void* stream);

/* Stages of one FISTA iteration, for per-kernel timing and profiling. */
typedef enum {
  OCT_STAGE_LAT_FWD = 0,    /* X1 = F_lat(z + mu (z - z_prev))          (eq. (4), (15)) */
  OCT_STAGE_NUFFT_FWD = 1,  /* W = H . KB-NUFFT_q(X1)                   (eq. (5)-(6))   */
  OCT_STAGE_NORMAL = 2,     /* W = F_lat(s.(Re F_lat^-1 W - y)) / N_lat (eq. (2), (7))  */
  OCT_STAGE_NUFFT_ADJ = 3,  /* X1 = NUFFT_q^H(conj(H) . W)              (eq. (3))       */
  OCT_STAGE_LAT_UPDATE = 4, /* v = x - delta F_lat^H X1                 (eq. (15))      */
  OCT_STAGE_PROX = 5,       /* z = prox(v) for the given penalty        (eq. (16))      */
  OCT_STAGE_NUFFT_NORMAL = 6 /* X1 = NUFFT_q^H(conj(H) . (H . KB-NUFFT_q(X1) residual spectrum)),
                                every pixel observed (eq. (2)-(7))                          */
} oct_stage;

/* Run one stage of a FISTA iteration on the plan's own workspace and solver
 * buffers (their contents are whatever earlier calls left, zero at first
 * use), with the kernels and launch shapes oct_mbir_solve uses.  For timing
 * and profiling only; y is read by OCT_STAGE_NORMAL (device measurement,
 * may be NULL for the others); penalty selects the prox (TV with 10 inner
 * steps, Haar with 3 levels).  On a plan whose every pixel is observed
 * (mask NULL or all ones) the solve's column stages are one:
 * OCT_STAGE_NUFFT_NORMAL, the forward columns, the residual spectrum
 * W_h/N_lat - F_lat(y)/N_lat (from the solver's stored F_lat(y)) and the
 * adjoint columns in one kernel per column pair (or the two pair kernels
 * when a pair's samples do not fit its registers); OCT_E_UNSUPPORTED on a
 * masked plan.  The other stages still run as named: OCT_STAGE_NUFFT_FWD
 * then writes the residual spectrum, and OCT_STAGE_NORMAL runs the general
 * seam.  Asynchronous. */
oct_status oct_run_stage(oct_plan_t plan, int32_t stage, int32_t penalty, const float* y, void* stream);

/* Direct (non-iterative) reconstructions of Sec. 3.1: the three images of
 * Figure 1 and the baseline of the sub-sampling study. */
typedef enum {
  OCT_DIRECT_AXIAL = 0,       /* "IFFT": per-A-scan depth transform, no dispersion
                                 compensation: the adjoint of the model restricted
                                 to lateral frequency zero (beta = 2k, no beam term),
                                 Omega = 0, applied to s . y                          */
  OCT_DIRECT_DISPERSION = 1,  /* the same with the dispersion phase of eq. (9)
                                 removed ("dispersion corrected")                    */
  OCT_DIRECT_ISAM = 2,        /* Phi^H (s . y): dispersion compensation and the ISAM
                                 resampling (eq. (5)); same as oct_adjoint            */
  OCT_DIRECT_INTERP_ISAM = 3  /* baseline: each A-scan's unobserved samples linearly
                                 interpolated in k from its observed ones (nearest
                                 observed value outside their range, zero if none),
                                 then Phi^H with every sample observed               */
} oct_direct_kind;

/* x = the direct reconstruction `kind` of the measurement y.
 * y: device float32 [batch][n_y][n_x][n_k] (read); x: device complex64
 * [batch][n_y][n_x][n_depth] (written).  Uses the plan's workspace (and, for
 * OCT_DIRECT_INTERP_ISAM, a filled-spectrum buffer the plan allocates on
 * first use: n_k * n_x * n_y * batch floats).  Asynchronous on `stream`.
 * Errors: OCT_E_INVALID (null pointer, unknown kind), OCT_E_NOMEM,
 * OCT_E_DEVICE. */
oct_status oct_direct(oct_plan_t plan, int32_t kind, const float* y, void* x, void* stream);

/* Normalised cross-correlation of magnitudes, eq. (17):
 *   r = sum (|x_i| - mean|x|)(|z_i| - mean|z|) / sqrt(sum (|x_i| - mean|x|)^2 sum (|z_i| - mean|z|)^2)
 * over the plan's image size, z the reference ("ground truth").  x, z: device
 * complex64 images (read).  Sums in FP64 on the device (two passes: means,
 * then centred sums, deterministic order); r_out: HOST double (written).
 * Synchronizes `stream`.  Errors: OCT_E_INVALID (null pointer; also when
 * either image has zero magnitude variance), OCT_E_DEVICE. */
oct_status oct_ncc(oct_plan_t plan, const void* x, const void* z, double* r_out, void* stream);

/* oct_ncc without a plan and without allocating: for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same sums and block count as oct_ncc, so
 * the result agrees with it to rounding of the final division.
 * x, z: device complex64 arrays of n elements (read); r_out: DEVICE double
 * (written): the NCC of eq. (17), NaN when either image has constant
 * magnitude.  n in 1..OCT_NCC_NOALLOC_MAX_N, else OCT_E_INVALID.
 * Scratch: a static device array of (3 * 1024 + 8) doubles (24.6 KB) per GPU,
 * held until the process ends and shared by every call on that GPU; it needs
 * no clearing (every read is of a value the same call wrote).  Calls that
 * overlap on one GPU (two streams, two threads) race on it: serialise them.
 * Asynchronous on `stream`; no allocation, no host synchronisation.
 * Errors: OCT_E_INVALID, OCT_E_DEVICE. */
#define OCT_NCC_NOALLOC_MAX_N ((int64_t)1 << 40)
oct_status oct_ncc_noalloc(const void* x, const void* z, int64_t n, double* r_out, void* stream);

/* Message for the last non-OK status returned to the calling thread. */
const char* oct_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* OCT_H */

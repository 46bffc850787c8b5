/*
 * fwi.h -- C-ABI of the MI355X (gfx950) k-space time-reversal gradient library.
 *
 * Method: Lucka, Perez-Liva, Treeby, Cox, "High Resolution 3D Ultrasonic
 * Breast Imaging by Time-Domain Full Waveform Inversion" (arXiv 2102.00755).
 *   - forward model  f = M A(u)^-1 s                      (Sec. 2.2, eq. USTmodel)
 *   - misfit         D = 1/2 || f - f^delta ||^2           (Sec. 2.3, eq. FWI)
 *   - gradient       dD/dc0 via adjoint + time reversal    (Sec. 2.3 eq. Gradc0,
 *                                                           Sec. 3.1 eq. TRBwdWave,
 *                                                           App. B, Algorithm 1)
 *   - encoding       s_hat = sum_i w_i s_i, w_i = +-1      (Sec. 3.2, App. E)
 *   - discretisation k-space pseudospectral scheme with split density and
 *                    PML                                    (App. B, eq. DisPartDev,
 *                                                           eq. DisPartDevSt)
 *
 * Conventions shared by every entry point
 *   - Grids are [nz][ny][nx], x fastest, spacing dx in all three axes.  The
 *     PML lies inside the grid (pml[a] cells at both ends of axis a).
 *   - Every array argument of a compute entry point is a DEVICE pointer on the
 *     handle's device, in the handle's precision ("real" = float when
 *     precision == 4, double when precision == 8), allocated and owned by the
 *     caller.  The library never frees or keeps caller pointers beyond a call.
 *   - Batched entry points take B contiguous problems: [B][...] arrays.
 *   - Calls are asynchronous on the given HIP stream (0 = null stream) unless
 *     a flag requests a check that reads a device flag back.
 *   - Return value: FWI_OK or one of the FWI_ERR_* codes; no exception or
 *     abort crosses this boundary.  A handle is not thread-safe; distinct
 *     handles may be used concurrently (on distinct streams).
 *   - Supported sizes: nx even with nx/2 in, and ny, nz in, the set
 *     {8, 12, 16, 24, 32, 40, 48, 56, 64, 80, 96, 112, 128, 160, 192, 224, 240,
 *      256, 320, 384, 448, 480, 512} (2-, 3-, 5-, 7-smooth lengths; the paper's
 *     PML-padded 480 x 480 x 256 grid among them); other sizes return
 *     FWI_ERR_UNSUPPORTED.
 */
#ifndef FWI_H_
#define FWI_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fwi_handle fwi_handle;
typedef struct ihipStream_t* fwi_stream_t; /* a hipStream_t */

enum {
  FWI_OK = 0,
  FWI_ERR_INVALID_ARG = 1,  /* bad shape/pointer/geometry, c outside [c_min,c_max] */
  FWI_ERR_UNSUPPORTED = 2,  /* grid size not in the supported FFT set */
  FWI_ERR_OOM = 3,          /* device allocation failed */
  FWI_ERR_NO_TAPE = 4,      /* backward without a forward that saved the tape */
  FWI_ERR_HIP = 5,          /* a HIP runtime call failed */
  FWI_ERR_UNSTABLE = 6      /* non-finite value detected in the result */
};

/* Flags of fwi_forward / fwi_gradient / fwi_backward. */
enum {
  FWI_SAVE_TAPE = 1,    /* forward keeps the dGamma tape for fwi_backward     */
  FWI_CHECK_INPUT = 2,  /* validate c in [c_min, c_max] (reads a flag back)   */
  FWI_CHECK_FINITE = 4, /* check outputs are finite (reads a flag back)       */
  FWI_TR_FINAL_STATE = 8, /* start the TR run from the final forward state
                             instead of the paper's zero interior           */
  FWI_GRAPH = 16,         /* capture one time step in a hipGraph and replay it
                             (step index read from device memory); results
                             are identical to eager launches                 */
  FWI_MEAN = 32,          /* fwi_gradient / fwi_backward: write the mean of the
                             B gradients, (1/B) sum_b G_b summed in FP64 in the
                             order b = 0..B-1, to ONE grid [nz][ny][nx]
                             (averaging of independent encoded realisations,
                             Sec. 3.2); misfit stays [B]                     */
  FWI_EXACT = 64          /* fwi_gradient: the exact discrete gradient dD/dc0
                             on Gamma instead of Alg. 1's TR gradient:
                             reverse-mode differentiation of every operation
                             of the forward iteration (PML included; with
                             absorption set, the dL/dc0 terms of App. A:
                             dp/dc0 = (2/c0) p + c0^2 (tau' A[d] - eta' B[s])),
                             from a history of dp/dc0 on Gamma stored by the
                             forward run (nt x |Gamma| values of the handle's
                             precision, allocated on first use: FWI_ERR_OOM).
                             The c0 of the source scaling is held fixed.
                             B = 1 only, without FWI_GRAPH, FWI_MEAN or
                             FWI_TR_FINAL_STATE (FWI_ERR_INVALID_ARG)        */
};

/* Scheme parameters (App. B).  dt = cfl dx / c_max in the paper (Sec. 4.1). */
typedef struct {
  int32_t nx, ny, nz;   /* grid (FFT) sizes                                   */
  double dx;            /* grid spacing [m]                                   */
  double dt;            /* time step [s]                                      */
  double c_ref;         /* k-space reference speed (paper: c_ref = c0^max)    */
  double c_min, c_max;  /* admissible sound-speed bounds [m/s]                */
  double rho0;          /* constant ambient density [kg/m^3]                  */
  int32_t pml[3];       /* PML thickness in cells along x, y, z (inside grid) */
  double pml_alpha;     /* PML strength: alpha = pml_alpha (c_ref/dx) (d/P)^4 */
  int32_t nt;           /* number of time steps N                             */
  int32_t precision;    /* 4 (float) or 8 (double)                            */
  int32_t batch;        /* maximum number of problems per batched call (>=1) */
} fwi_params;

/* Geometry: transducer voxels and the region of interest (host arrays, read
 * only during fwi_create).  Sources and receivers are point transducers
 * snapped to voxels (Sec. 4.1); Gamma is the region where c0 is sought and
 * dGamma the layer of Gamma voxels whose pressure is taped for the time
 * reversal (Sec. 3.1, Sec. 4.2).  Duplicate source voxels, duplicate receiver
 * voxels, transducers inside Gamma, dGamma voxels outside Gamma, and any of
 * these inside the PML are rejected with FWI_ERR_INVALID_ARG. */
typedef struct {
  int32_t n_src;
  const int32_t* src_ijk;        /* host [n_src][3] = (ix, iy, iz)           */
  int32_t n_rec;
  const int32_t* rec_ijk;        /* host [n_rec][3]                          */
  const uint8_t* gamma_mask;     /* host [nz][ny][nx], nonzero inside Gamma  */
  const uint8_t* boundary_mask;  /* host [nz][ny][nx], nonzero on dGamma     */
} fwi_geometry;

/* Create a handle on HIP device `device`: validates params and geometry,
 * builds the operator tables (wavenumbers, kappa inputs, staggering phases,
 * PML profiles: App. B) and allocates the whole workspace for `batch`
 * problems (fields, spectra, tape).  *out is set to NULL on failure. */
int fwi_create(const fwi_params* params, const fwi_geometry* geom, int device,
               fwi_handle** out);

/* Release the handle and all device memory it owns.  NULL is allowed. */
void fwi_destroy(fwi_handle* h);

/* Device bytes fwi_create would allocate for these params/geometry (the
 * admission query of a serving loop).  Host-only; returns 0 on invalid input. */
int64_t fwi_workspace_bytes(const fwi_params* params, const fwi_geometry* geom);

/* Rademacher encoding weights (Sec. 3.2: w_i = +-1 with equal probability):
 * w_out[i] = +1 if the top bit of the i-th output of SplitMix64 (Steele, Lea,
 * Flood 2014) seeded with `seed` is 0, else -1.  Host array, n >= 0. */
int fwi_rademacher(uint64_t seed, int32_t n, int8_t* w_out);

/* Delays of delayed source encoding (Sec. 3.2, eq. DelaySE): source i fires
 * d_i tau later, d_i ~ U[0,1).  d_i is the i-th uniform of the same SplitMix64
 * stream as fwi_rademacher, taken at counter n + i (so weights and delays of
 * one seed are independent): d_i = (z >> 11) * 2^-53 with z its output, and
 * out[i] = floor(d_i * tau_steps + 1/2) whole time steps, to be passed to
 * fwi_set_delays; the handle then runs nt = (signal length) + tau_steps steps
 * and the caller's observed data are the delayed-encoded data.  Host arrays,
 * n >= 0, tau_steps >= 0. */
int fwi_delays(uint64_t seed, int32_t n, int32_t tau_steps, int32_t* out);

/* Delayed source encoding (Sec. 3.2, eq. DelaySE): source i of problem b
 * fires its signal delays[b][i] whole steps late, i.e. the injection of step n
 * uses src_sig[b][n - delays[b][i]][i] (zero for n < delays[b][i]); the
 * signals passed to fwi_forward / fwi_gradient stay unshifted.
 *   delays  host [B][n_src] int32, each in [0, nt); copied into the handle
 *           (rows b >= B are zero).  B = 0 (delays may be NULL) switches
 *           delays off.
 * Applies to every later fwi_forward and fwi_gradient of the handle (the
 * adjoint and TR simulations inject no sources).  Synchronises the device
 * first, so no call of the handle may be in flight on another thread.
 * FWI_ERR_INVALID_ARG (nothing changed) for a NULL handle, B outside
 * [0, batch], a NULL array with B > 0 or a delay outside [0, nt). */
int fwi_set_delays(fwi_handle* h, int32_t B, const int32_t* delays);

/* Forward simulation (Alg. 1 forward iteration) of B problems:
 *   c        [B][nz][ny][nx]  sound speed, in [c_min, c_max]
 *   src_sig  [B][nt][n_src]   source signals s_i(t_n)
 *   w        [B][n_src]       int8 weights in {-1, 0, +1}; encoded source
 *                             s_hat = sum_i w_i s_i (Sec. 3.2, tau = 0)
 *   traces   [B][nt][n_rec]   output f^n = M p^{n+1}, n = 0..nt-1
 * With FWI_SAVE_TAPE the dGamma pressure history is kept in the handle for
 * fwi_backward (B must then be <= batch). */
int fwi_forward(fwi_handle* h, int32_t B, const void* c, const void* src_sig,
                const int8_t* w, void* traces, int32_t flags, fwi_stream_t stream);

/* Encoded TR gradient (Alg. 1) of B problems: forward with tape, residual
 * r = f - f^delta, misfit D = 1/2 sum r^2 (FP64), then the interleaved
 * adjoint and time-reversal simulations accumulating
 *   G = sum_j 2/c0^3 p_adj^(j) (p_tr^(j) - 2 p_tr^(j+1) + p_tr^(j+2))  on Gamma.
 *   obs      [B][nt][n_rec]   observed (encoded) data f^delta
 *   misfit   [B] double       output D
 *   grad     [B][nz][ny][nx]  output gradient, zero outside Gamma ([nz][ny][nx]:
 *                             their mean, with FWI_MEAN)
 * Three wave simulations per problem (Sec. 3.1). */
int fwi_gradient(fwi_handle* h, int32_t B, const void* c, const void* src_sig,
                 const int8_t* w, const void* obs, double* misfit, void* grad,
                 int32_t flags, fwi_stream_t stream);

/* Backward of the forward map c -> traces (the adjoint of Sec. 2.3 through
 * time reversal): given residual = dL/df [B][nt][n_rec], returns
 * grad = (df/dc)^T residual restricted to Gamma, recomputing the forward field
 * by time reversal from the tape saved by the last fwi_forward with
 * FWI_SAVE_TAPE (same B, same c).  misfit[b] = 1/2 ||residual_b||^2.
 * Two wave simulations per problem.  FWI_ERR_NO_TAPE without a saved tape. */
int fwi_backward(fwi_handle* h, int32_t B, const void* c, const void* residual,
                 double* misfit, void* grad, int32_t flags, fwi_stream_t stream);

/* One spectral derivative (eq. DisPartDevSt) of a field, for parity tests:
 * out = Re F^-1 { i k_a kappa exp(sign i k_a dx/2) F{in} }, a in {0,1,2} =
 * x, y, z, sign = +1 or -1.  in/out [nz][ny][nx] device, may not alias. */
int fwi_derivative(fwi_handle* h, const void* in, void* out, int32_t axis, int32_t sign,
                   fwi_stream_t stream);

/* Launch tuning of a handle: the row segment, in bytes, of the tiles of the
 * y passes, of the z pass of d- (Z1) and of the z pass of d+ (Z2), each 64 or
 * 128; and the radix plan of the transforms of the y passes, of Z1, of Z2 and
 * of the velocity and density x passes (length nx/2), each 0 or 1:
 *   plan 0: the odd radices (7, 5, 3) first, then radix-8 stages with the
 *           smaller power-of-two stage last (e.g. 224 = 7 * 8 * 4);
 *   plan 1: the same radices with the power-of-two stages in reverse order
 *           (224 = 7 * 4 * 8); lengths whose two plans coincide run plan 0.
 * The tile width changes only which threads compute which columns, not the
 * arithmetic: results are bit-identical across tile widths.  The two radix
 * plans compute the same DFT in a different order of operations: results
 * agree to rounding (both are parity-tested).  New handles start from the
 * build's defaults (measured fastest at 448x448x224);
 * paper_2102_00755_amd.autotune measures the alternatives per grid. */
typedef struct {
  int32_t y_tile_bytes;
  int32_t zm_tile_bytes;
  int32_t zp_tile_bytes;
  int32_t y_plan;
  int32_t zm_plan;
  int32_t zp_plan;
  int32_t x_plan;
} fwi_tuning;

/* Read the handle's tuning into *out. */
int fwi_get_tuning(const fwi_handle* h, fwi_tuning* out);

/* Set the tuning used by subsequent calls on the handle (not by calls already
 * enqueued).  FWI_ERR_INVALID_ARG (tuning unchanged) for other values. */
int fwi_set_tuning(fwi_handle* h, const fwi_tuning* t);

/* Power-law absorption and dispersion (Sec. 2.1, the operator L of the
 * pressure-density relation eq. PreDenRel; Sec. 3.1 for time reversal in
 * absorbing media).  While set, every simulation of the handle uses
 *   p = c0^2 (s + tau A[d] - eta B[s]),  s = sum_xi rho_xi,
 *   d = rho0 sum_xi d-_xi v_xi,  A = F^-1 |k|^{y-2} F,  B = F^-1 |k|^{y-1} F
 *   (both multipliers 0 at k = 0),
 *   tau = -2 alpha0 c0^{y-1},  eta = 2 alpha0 c0^y tan(pi y / 2),
 * in place of p = c0^2 s: fwi_forward, fwi_gradient, fwi_backward and the
 * batched gradient.  The adjoint simulation uses the same lossy step; the TR
 * simulation switches the sign of tau when tr_flip != 0 (Sec. 3.1) and keeps
 * it otherwise; the gradient keeps the form of Alg. 1 (2 / c0^3 times the
 * second time difference of the TR pressure against the adjoint pressure,
 * without the dL/dc0 terms of App. A); fwi_gradient with FWI_EXACT returns
 * the exact discrete gradient, which carries them.
 *   alpha0        Np (rad/s)^-y m^-1 (uniform), >= 0 and finite
 *   y             power-law exponent, 0 < y < 2, y != 1
 *   alpha0_field  NULL, or a device array [nz][ny][nx] of the handle's
 *                 precision holding alpha0 per voxel (then alpha0 is unused
 *                 except for alpha0 == 0 && alpha0_field == NULL, which
 *                 switches absorption off); read by every later call, so it
 *                 must stay allocated while absorption is set (the caller owns it)
 * The lossy step forms A[d] in its velocity-divergence z pass and replaces
 * the fused X2 pass by five launches (density update, forward y, absorption
 * z pass of B[s], inverse y, equation of state); FWI_GRAPH replays it as a
 * step graph like the lossless step; FWI_TR_FINAL_STATE is rejected with
 * FWI_ERR_INVALID_ARG.  The first call that switches absorption on allocates
 * batch x |Gamma| values and two half spectra per problem of device memory
 * (FWI_ERR_OOM on failure).  Any call invalidates the saved tape.  Errors:
 * FWI_ERR_INVALID_ARG (nothing changed) for a NULL handle, alpha0 < 0 or not
 * finite, or y outside the range. */
int fwi_set_absorption(fwi_handle* h, double alpha0, double y, const void* alpha0_field, int32_t tr_flip);

/* Pass kinds of one time step, for fwi_timing_* (one kernel symbol each). */
enum {
  FWI_PASS_Y_FWD = 0,    /* forward y-FFT                                     */
  FWI_PASS_Y_INV = 1,    /* inverse y-FFT                                     */
  FWI_PASS_Z_PLUS = 2,   /* z-FFT, k-space multiply for d+, v_z update        */
  FWI_PASS_Z_MINUS = 3,  /* z-FFT, k-space multiply for d- (3 -> 3 fields)    */
  FWI_PASS_X_VEL = 4,    /* C2R, v_x update, R2C                              */
  FWI_PASS_X_DEN_FWD = 5,  /* C2R, density/EOS/sources/sensors/tape, R2C       */
  FWI_PASS_X_DEN_PAIR = 6, /* adjoint + TR density passes with gradient        */
  FWI_PASS_Y_VEL_Q = 7,  /* inverse y-FFT of Q (Z2) with the v_y update        */
  FWI_PASS_COUNT = 8
};

/* Sampled timing of the pass launches, for roofline measurement: when
 * every > 0, every `every`-th time step of subsequent forward / gradient /
 * backward calls brackets each pass launch with two HIP events on the call's
 * stream; the call then synchronises its stream once at its end to collect
 * them.  every = 0 disables sampling. */
int fwi_timing_enable(fwi_handle* h, int32_t every);

/* Accumulated samples of one pass kind since the last read (then reset):
 * number of sampled launches, their summed duration [ms] and the summed
 * algorithmic HBM bytes of those launches (the bytes the pass must move:
 * spectra, fields, sound speed, tape, ring and accumulator, counted once). */
int fwi_timing_read(fwi_handle* h, int32_t pass, int64_t* launches, double* total_ms, double* total_bytes);

/* ---- Outer loop: stochastic L-BFGS (App. D, Algorithm 2) ------------------
 * Device vector primitives of the SLBFGS iteration over the unknowns on
 * Gamma; the gradient itself comes from fwi_gradient.  Vectors are device
 * arrays of n reals in the given precision (4 float, 8 double), owned by the
 * caller; all calls are asynchronous on the stream. */

/* Number of Gamma voxels (length of a Gamma-compact vector) of the handle. */
int fwi_gamma_size(const fwi_handle* h, int64_t* n);

/* compact[k] = full[k-th Gamma voxel in [z][y][x] order] (gather), or
 * full[k-th Gamma voxel] = compact[k] leaving the rest of full unchanged
 * (scatter).  full is one [nz][ny][nx] grid in the handle's precision. */
int fwi_gamma_gather(fwi_handle* h, const void* full, void* compact, fwi_stream_t stream);
int fwi_gamma_scatter(fwi_handle* h, const void* compact, void* full, fwi_stream_t stream);

/* L-BFGS history of at most m pairs (s, y) of length-n vectors (the buffers S
 * and Y of Algorithm 2), allocated on `device`; *out NULL on failure
 * (FWI_ERR_OOM).  Not thread-safe; one history per optimisation. */
typedef struct fwi_lbfgs fwi_lbfgs;
int fwi_lbfgs_create(int64_t n, int32_t m, int32_t precision, int32_t device, fwi_lbfgs** out);
void fwi_lbfgs_destroy(fwi_lbfgs* L);

/* Append the pair (s, y) (copied), dropping the oldest pair when m are
 * stored, and set rho = 1 / y^T s (FP64 reduction in a fixed order: results
 * are deterministic).  No curvature check: the pair is used as given. */
int fwi_lbfgs_push(fwi_lbfgs* L, const void* s, const void* y, fwi_stream_t stream);

/* r = H g, H the L-BFGS inverse-Hessian approximation of the stored pairs with
 * initial matrix h0 I (two-loop recursion: Nocedal & Wright, Numerical
 * Optimization, Algorithm 7.4).  r may alias g.  Dot products accumulate in
 * FP64 in a fixed order; their scalars stay in device memory. */
int fwi_lbfgs_apply(fwi_lbfgs* L, const void* g, void* r, double h0, fwi_stream_t stream);

/* fwi_lbfgs_apply for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same two-loop recursion, bit-identical results, but its scratch (the
 * alpha_j, the second-loop coefficient and the dot-product partial sums) is
 * a static device array of the library, sized for FWI_NOALLOC_MAX_PAIRS
 * pairs, instead of memory owned by the history; the call makes no
 * allocation (no hipMalloc, hipFree or allocating library routine).  The
 * history itself still comes from fwi_lbfgs_create (set-up time).
 * Each device has ONE such array, shared by every call on that device and
 * kept until the process ends: calls of this entry point that overlap on one
 * device (on different streams or threads) race and give wrong results; order
 * them on one stream.  FWI_ERR_INVALID_ARG (nothing launched) for a NULL
 * argument or a history of more than FWI_NOALLOC_MAX_PAIRS pairs (its m). */
enum { FWI_NOALLOC_MAX_PAIRS = 256 };
int fwi_lbfgs_apply_noalloc(fwi_lbfgs* L, const void* g, void* r, double h0, fwi_stream_t stream);

/* Number of stored pairs (host bookkeeping, no device access). */
int fwi_lbfgs_count(const fwi_lbfgs* L, int32_t* count);

/* y = a x + b y (x may be NULL: y = b y); with b = 0, y is not read. */
int fwi_vec_axpby(int64_t n, double a, const void* x, double b, void* y, int32_t precision, fwi_stream_t stream);

/* x = max(min(x, hi), lo): the projection onto bound constraints (Alg. 2). */
int fwi_vec_clip(int64_t n, void* x, double lo, double hi, int32_t precision, fwi_stream_t stream);

/* Squared-slowness parametrisation u = 1 / c0^2 (Sec. 2.4 preconditioning):
 * mode 0: out = 1 / in^2 (c0 -> u); mode 1: out = 1 / sqrt(in) (u -> c0);
 * mode 2: out = -aux^3 in / 2, the gradient with respect to u from the
 * gradient `in` with respect to c0 at c0 = aux (dc0/du = -c0^3 / 2). */
int fwi_vec_sqslowness(int64_t n, int32_t mode, const void* in, const void* aux, void* out, int32_t precision,
                       fwi_stream_t stream);

/* ---- Grid transfers of the coarse-to-fine scheme (Sec. 2.4, App. C) -------- */

/* Fourier interpolation of the real field `in` on the coarse handle's grid to
 * `out` on the fine handle's grid (both [nz][ny][nx] device arrays of the
 * handles' common precision; the grids must cover the same box: n_a dx equal
 * per axis, each fine size >= the coarse one).  The coarse DFT is embedded in
 * the fine frequency grid (zeros elsewhere; the Nyquist bin of an even coarse
 * axis split in halves over +-N/2) and transformed back; window = 1 multiplies
 * by the separable Blackman window of the coarse band, 0.42 + 0.5 cos(pi k/K)
 * + 0.08 cos(2 pi k/K), K = N_coarse/2 per axis (App. C smoothing), window = 0
 * by nothing.  Uses the handles' scratch spectra (a later fwi_backward needs a
 * new FWI_SAVE_TAPE forward).  Same device for both handles. */
int fwi_interp_fourier(fwi_handle* coarse, fwi_handle* fine, const void* in, void* out, int32_t window,
                       fwi_stream_t stream);

/* Band-limited resampling of time series in [nt_in][n_ch] (step dt_in) to
 * out [nt_out][n_ch] (step dt_out), with a low-pass cut-off f_cut [Hz]: the
 * Kaiser-windowed sinc
 *   out[m] = scale sum_n in[n] 2 f_cut dt_in sinc(2 f_cut tau) I0(beta sqrt(1 - (tau/t_window)^2)) / I0(beta),
 *   tau = m dt_out - n dt_in, terms with |tau| > t_window omitted
 * (App. C: sources and data to the coarse time step; data with
 * scale = eta^(d-1)).  Device arrays; FP64 accumulation. */
int fwi_resample_time(int32_t nt_in, int32_t n_ch, const void* in, double dt_in, int32_t nt_out, double dt_out,
                      double f_cut, double beta, double t_window, double scale, void* out, int32_t precision,
                      fwi_stream_t stream);

/* Human-readable text of a status code (static storage). */
const char* fwi_status_string(int status);

/* Last error detail recorded on this thread (static storage, may be ""). */
const char* fwi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FWI_H_ */

/*
 * nufftct — NUFFT projector from a 3D volume to its radially sampled
 * first-derivative Radon space, and the exact adjoint, on one AMD MI355X (gfx950).
 *
 * The forward operator is module 1 of the NUFFT cone-beam forward projector
 * (Section 2, first of its three steps; Section 2.2.1; Section 2.4.1,
 * eq 2.16-2.18):
 *
 *   1. scale the volume by the deapodization factors and zero-pad it to K^3
 *      (the diagonal P of eq 2.11),
 *   2. unnormalised oversampled 3D FFT (F of eq 2.11),
 *   3. J^3 Kaiser-Bessel or min-max interpolation onto the points
 *      omega_p (T_sparse of eq 2.11; the paper's "NUFFT"),
 *   4. optionally, per radial line, the derivative factor i*r and a 1D
 *      inverse DFT (eq 2.17-2.18), giving derivative-Radon values.
 *
 * The adjoint ("NUFFT transpose", Introduction; Section 2.3) applies the
 * conjugate transposes in reverse order: radial DFT with factor -i*r, J^3
 * spreading, unnormalised inverse FFT, crop and deapodization.
 *
 * Conventions (readings where the paper is silent):
 *   volume     x[n0][n1][n2], n2 fastest, N^3 complex values; centred index
 *              m = n - N/2; N even.
 *   transform  X(omega) = sum_n x[n] exp(-i omega . m), omega in rad/voxel.
 *   points     radial plans: line l has unit direction nhat_l (3 doubles) and
 *              N_r samples r_c = (c - N_r/2) * (2 pi / N_r), c = 0..N_r-1;
 *              omega[l*N_r + c] = r_c * nhat_l.  Point plans take omega
 *              directly (M x 3 doubles, row-major).
 *   kernel     KB: psi(u) = I0(beta sqrt(1-(2u/J)^2))/I0(beta), beta <= 0
 *              selects 2.34*J; deapodization s(m) = 1/Psi(m/K) with Psi the
 *              kernel's continuous Fourier transform.  MINMAX_KB: per-axis
 *              min-max coefficients c = T^-1 r with the same scaling s(m).
 *   neighbours per axis t = omega_d / (2 pi / K) in FP64, k0 = floor(t - J/2),
 *              taps k0+1 .. k0+J (wrapped mod K).
 *   radial     D[l][j] = (1/N_r) sum_c f_c G[l][c] exp(+i r_c (j - N_r/2)),
 *              f_c = i r_c (f_0 = 0) with DERIV, f_c = 1 without.
 *   complex    interleaved (re, im); FP32 plans use complex64 (2 x float),
 *              FP64 plans complex128 (2 x double).
 *
 * Memory and threads: all data pointers passed to forward/adjoint are DEVICE
 * pointers owned by the caller, contiguous, and must not alias each other.
 * The plan owns every table, the K^3 workspace and the point permutation.
 * Calls are asynchronous and stream-ordered on the given stream (a
 * hipStream_t passed as void*, NULL = the null stream); plan creation is the
 * only blocking call.  One plan is used by one stream at a time (it holds a
 * single workspace); separate plans are independent.  Nothing throws across
 * this interface: every entry point returns a status code, and
 * nufftct_last_error() returns this thread's message for the last failure.
 * Device faults of asynchronous kernels surface at the caller's next
 * synchronisation.
 */
#ifndef NUFFTCT_H
#define NUFFTCT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nufftct_plan nufftct_plan;
typedef struct nufftct_batch nufftct_batch;
typedef struct nufftct_umbrella nufftct_umbrella;
typedef struct nufftct_grangeat nufftct_grangeat;

/* status codes */
#define NUFFTCT_OK 0
#define NUFFTCT_EINVAL 1       /* bad argument: sizes, null pointer, precision */
#define NUFFTCT_ENOMEM 2       /* device or host allocation failed */
#define NUFFTCT_EHIP 3         /* HIP runtime or launch error */
#define NUFFTCT_EUNSUPPORTED 4 /* e.g. a grid size with a prime factor > 5 */

/* interpolation kernels */
#define NUFFTCT_KERNEL_KB 0
#define NUFFTCT_KERNEL_MINMAX_KB 1

/* arithmetic precision of the whole path */
#define NUFFTCT_FP32 0 /* complex64 data; tables built in FP64 and rounded once */
#define NUFFTCT_FP64 1 /* complex128 data, FP64 throughout */

/* flags for forward / adjoint */
#define NUFFTCT_RADIAL 1 /* apply the per-line radial (inverse) DFT stage */
#define NUFFTCT_DERIV 2  /* with RADIAL: include the i*r derivative factor */
#define NUFFTCT_DERIV_RADIAL 3
/* adjoint: bitwise reproducible spreading.  The FP32 path always spreads in
 * fixed point (integer sums do not depend on the order of the atomic adds);
 * with this flag the FP64 form does too (64-bit words, scale 2^62 / (vmax B)
 * per task), instead of FP64 atomic adds whose rounding follows their order.
 * Accepted, and without effect, by the forward operator. */
#define NUFFTCT_DETERMINISTIC 4

/* stages for nufftct_stage (one stage of the path, for testing and profiling) */
#define NUFFTCT_STAGE_PAD_FFT 0   /* vol[N^3]  -> grid[K^3] centred spectrum (F1+F2) */
#define NUFFTCT_STAGE_INTERP 1    /* grid[K^3] -> G[M], line order (F3)             */
#define NUFFTCT_STAGE_RADIAL 2    /* G[M]      -> D[M] (F4; flags select DERIV)       */
#define NUFFTCT_STAGE_RADIAL_ADJ 3 /* D[M]     -> G~[M] (A4)                          */
#define NUFFTCT_STAGE_SPREAD 4    /* G~[M]     -> grid[K^3] (A3)                     */
#define NUFFTCT_STAGE_IFFT_CROP 5 /* grid[K^3] -> vol[N^3] (A2+A1)                   */

/*
 * Create a plan for explicit points (Section 2.1.3, eq 2.8-2.11: x~ = T x at
 * arbitrary non-uniform points).
 *   N          volume edge (even, >= 2)
 *   K          oversampled grid edge (even, >= N; prime factors 2, 3, 5;
 *              8 <= K <= 1024)
 *   J          taps per axis, 2 <= J <= 8, J <= K
 *   kernel     NUFFTCT_KERNEL_KB or NUFFTCT_KERNEL_MINMAX_KB
 *   beta       KB shape; <= 0 selects 2.34*J
 *   precision  NUFFTCT_FP32 or NUFFTCT_FP64
 *   points     HOST pointer, M x 3 doubles (omega in rad/voxel); copied
 *   M          number of points, 1 <= M < 2^31
 *   n_r        0, or the radial line length when the points form lines of
 *              n_r samples (enables NUFFTCT_RADIAL; M % n_r == 0, n_r even)
 *   stream     stream for the plan's uploads (NULL = null stream)
 * On success *out receives the plan; on failure *out is NULL.
 * FP32 plans take two points whose FP64 frequencies agree to 1e-12
 * (relative) and share their first tap cell as one frequency: one
 * interpolation gives both outputs, and the adjoint spreads the sum of their
 * two values with one set of weights (radial lines in opposite directions
 * sample almost every frequency twice).  FP64 plans treat every point alone.
 */
int nufftct_plan_create(nufftct_plan** out, int64_t N, int64_t K, int J, int kernel,
                        double beta, int precision, const double* points, int64_t M,
                        int64_t n_r, void* stream);

/*
 * Create a plan for radial lines (Section 2.1.1, eq 2.1; Section 2.2.1):
 * n_lines unit directions (HOST pointer, n_lines x 3 doubles, copied), each
 * line carrying n_r samples r_c = (c - n_r/2)(2 pi/n_r).  The device forms
 * omega = r_c * nhat_l itself in FP64.  n_r even, 4 <= n_r <= 1024.  Other
 * arguments as nufftct_plan_create.
 */
int nufftct_plan_create_radial(nufftct_plan** out, int64_t N, int64_t K, int J, int kernel,
                               double beta, int precision, const double* dirs,
                               int64_t n_lines, int64_t n_r, void* stream);

/*
 * Autotune the tiling of radial plans with these parameters: builds candidate
 * plans (tile edge 16 or 8 cells x 1024..16384 points per task), times one
 * forward + adjoint (flags as for nufftct_forward) of each on `stream`, and
 * records the fastest in a process-wide table that every later plan creation
 * with the same (N, K, J, kernel, precision, n_lines, n_r) and the same
 * direction coordinates (compared by a hash of their bytes) uses.  With the
 * environment variable NUFFTCT_TUNE_CACHE naming a file, results are appended
 * there and read back by later processes.  NUFFTCT_TILE / NUFFTCT_MAXPTS in the
 * environment override the table.  Blocking; allocates temporary buffers.
 * Outputs (any may be NULL): the chosen tile edge, points per task and the
 * measured milliseconds per forward + adjoint.
 */
int nufftct_autotune_radial(int64_t N, int64_t K, int J, int kernel, double beta, int precision,
                            const double* dirs, int64_t n_lines, int64_t n_r, int flags,
                            int* best_tile, int* best_max_pts, double* best_ms, void* stream);

/*
 * Forward operator: vol (device, N^3 complex) -> out (device, M complex, line
 * order p = l*n_r + c).  flags: 0 = plain NUFFT values X^(omega_p);
 * NUFFTCT_RADIAL adds the radial inverse DFT; NUFFTCT_DERIV_RADIAL adds the
 * derivative factor too (derivative-Radon values).
 */
int nufftct_forward(nufftct_plan* plan, const void* vol, void* out, int flags, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the forward
 * operator of nufftct_forward, same arguments and results, with its workspace
 * (the K^3 spectrum grid and, with NUFFTCT_RADIAL, the M values ahead of the
 * radial stage) in one static device array of 64 MiB that the library holds
 * on every GPU it runs on until the process ends, instead of the plan's.  The
 * call allocates nothing.  Plans whose workspace exceeds 64 MiB (K^3 x 8 bytes
 * for FP32 plus M x 8 with NUFFTCT_RADIAL; twice that for FP64) are rejected
 * with NUFFTCT_EINVAL.  Every call on a GPU shares that GPU's array, which
 * keeps the last call's contents: calls that overlap on one GPU (different
 * streams, or host threads) race and must be serialised by the caller.
 */
int nufftct_forward_noalloc(nufftct_plan* plan, const void* vol, void* out, int flags,
                            void* stream);

/*
 * Adjoint (exact conjugate transpose of nufftct_forward with the same flags):
 * in (device, M complex) -> vol (device, N^3 complex, overwritten).  With
 * NUFFTCT_DETERMINISTIC in flags the result is bitwise reproducible in both
 * precisions (the FP32 path always is).
 */
int nufftct_adjoint(nufftct_plan* plan, const void* in, void* vol, int flags, void* stream);

/*
 * Direct reconstruction from radially sampled first-derivative Radon data
 * (Section 2.3: the image -> Radon step inverted by a Fourier-domain ramp
 * filter and the NUFFT transpose; the Introduction's R^2 ramp of the 3D
 * parallel geometry).  With the 3D inverse Fourier transform written over
 * whole lines through the origin, every direction of the sphere taken once,
 *     x(m) = 1/(2 (2 pi)^3) int_{S^2} int r^2 X(r n) exp(i r n.m) dr dOmega,
 * the ramp r^2 is conj(f_c) f_c of the derivative factor, so
 *     vol = 1/(8 pi^2) * A^H diag(w) in,
 * A^H the adjoint with NUFFTCT_DERIV_RADIAL and w the per-line quadrature
 * weights of the directions (set with nufftct_set_line_weights).
 *
 * nufftct_radial_quadrature: weights for a product grid of azimuths phi
 * (periodic, any order of increasing values) and increasing polar angles
 * theta, lines ordered [phi][theta] (the layout of the radial directions):
 * w[a*n_theta + b] = dphi_a * dtheta_b * sin(theta_b), dphi_a half the
 * periodic distance between phi_a's neighbours, dtheta_b the trapezoid
 * weight on [theta_0, theta_last] (2 for a single polar angle).  HOST arrays
 * (w: n_phi * n_theta doubles, caller-owned); no device work.  Errors: EINVAL
 * (NULL array, a count < 1, non-finite values, theta not increasing).
 *
 * nufftct_set_line_weights: copies n_lines HOST doubles into the plan
 * (blocking; the plan owns the copy).  EINVAL: NULL, non-radial plan,
 * non-finite weight; ENOMEM.
 *
 * nufftct_reconstruct: in (device, M complex derivative-Radon values, line
 * order) -> vol (device, N^3 complex, overwritten); stream-ordered.  EINVAL:
 * NULL or aliasing buffers, non-radial plan, no weights set.
 */
int nufftct_radial_quadrature(const double* phi, int64_t n_phi, const double* theta,
                              int64_t n_theta, double* w);
int nufftct_set_line_weights(nufftct_plan* plan, const double* w, void* stream);
int nufftct_reconstruct(nufftct_plan* plan, const void* in, void* vol, void* stream);

/*
 * Run one stage of the path (NUFFTCT_STAGE_*) from `in` to `out` (device
 * pointers of the sizes listed with each stage).  STAGE_SPREAD overwrites all
 * K^3 cells of `out`.  Used by the stage-parity tests and by profiling.
 */
int nufftct_stage(nufftct_plan* plan, int stage, const void* in, void* out, int flags,
                  void* stream);

/* Destroy a plan and free everything it owns (never the caller's buffers). */
int nufftct_plan_destroy(nufftct_plan* plan);

/* Plan introspection: sizes of the plan (any pointer may be NULL). */
int nufftct_plan_info(const nufftct_plan* plan, int64_t* N, int64_t* K, int* J,
                      int64_t* M, int64_t* n_r, int* precision, int64_t* workspace_bytes);

/*
 * The plan's tiling of the grid for interpolation and spreading: the tile
 * edge in grid cells and the largest number of points per task (from the
 * autotuner's table, the environment, or the defaults; see
 * nufftct_autotune_radial).  Either pointer may be NULL.
 */
int nufftct_plan_tiling(const nufftct_plan* plan, int* tile, int* max_pts);

/* timing slot of the kernel that merges the spread's per-task halo tiles into the grid */
#define NUFFTCT_TIMING_MERGE 6

/*
 * Per-stage timing with HIP events recorded on the call's stream.
 * nufftct_set_timing(plan, 1) starts accumulating; nufftct_get_stage_times
 * synchronises on the recorded events and writes, for each slot s in 0..n-1
 * (NUFFTCT_STAGE_* order, then NUFFTCT_TIMING_MERGE; at most 8 slots), the
 * summed milliseconds to ms[s] and the number of timed launches to count[s]
 * (either may be NULL), then resets.  Slots INTERP, RADIAL, RADIAL_ADJ,
 * SPREAD and MERGE each time exactly one kernel; PAD_FFT and IFFT_CROP time
 * their three FFT-pass kernels together.
 */
int nufftct_set_timing(nufftct_plan* plan, int enable);
int nufftct_get_stage_times(nufftct_plan* plan, double* ms, int64_t* count, int n);

/*
 * Radial -> umbrella resampling of the derivative-Radon space, method 2 of
 * Section 2.1.3 (eq 2.15 with T_sparse2 the identity): step 2 of the
 * forward projector (Section 2), from the radial pattern (eq 2.1) that the
 * projector produces to the planes through the source positions of a
 * circular cone-beam scan (the umbrella pattern, Figure 2.2).
 *
 * Geometry (voxel units): source circle of radius source_radius in the
 * z = 0 plane, lambda_k = 2 pi k / n_proj; flat detector at source_detector
 * from the source, perpendicular to the central ray, side detector_side,
 * axes u = (-sin lambda, cos lambda, 0), v = (0, 0, 1).  Sample (k, i, j)
 * is the plane through the source and the detector line
 * u cos(alpha_i) + v sin(alpha_i) = t_j, alpha_i = pi i / n_alpha,
 * t_j = (j - n_t/2) detector_side / n_t: normal nhat = normalised
 * (e x q), e the line's direction, q from the source to the line's foot;
 * rho = nhat . source.  Its (theta, phi) = (acos nhat_z, atan2 mod 2 pi).
 *
 * Interpolation: the radial grid phi_a = 2 pi a / n_phi, theta_b = theta0 +
 * b dtheta, rho_j = j - n_r/2 is uniform in index space; per axis the J taps
 * k0+1..k0+J, k0 = floor(t - J/2), weights sinc(u) psi(u) normalised over
 * the taps (psi the Kaiser-Bessel window of width J, beta = 4J/3).  phi
 * wraps; theta and rho taps off the grid contribute nothing.
 *
 * radial (device): n_phi * n_theta * n_r complex, layout [phi][theta][rho]
 * (the projector's output for the (phi, theta) line grid).  out (device):
 * n_proj * n_alpha * n_t complex, layout [k][i][j].  Complex64 for FP32,
 * complex128 for FP64.  Create is host-only (no device memory).  Errors:
 * EINVAL (counts < 1, products >= 2^31, non-positive or non-finite
 * distances, J outside [2, 8], NULL or aliasing buffers), EUNSUPPORTED (weight
 * fit), EHIP (launch).
 */
int nufftct_umbrella_create(nufftct_umbrella** out, int64_t n_proj, int64_t n_alpha, int64_t n_t,
                            double source_radius, double source_detector, double detector_side,
                            int64_t n_phi, int64_t n_theta, double theta0, double dtheta,
                            int64_t n_r, int J, int precision, void* stream);
int nufftct_umbrella_resample(nufftct_umbrella* u, const void* radial, void* out, void* stream);
int nufftct_umbrella_destroy(nufftct_umbrella* u);

/*
 * Radial -> umbrella resampling, method 1 of Section 2.1.3 (eq 2.11:
 * x~ = T_sparse F P F^-1 x): the ideal interpolator of eq 2.8 (a periodic
 * sinc per axis, eq 2.2-2.7) computed as an oversampled NUFFT in the
 * (phi, theta, rho) index space of the radial grid.  Same scan geometry,
 * radial grid, target index coordinates and layouts as method 2 above;
 * nufftct_umbrella_resample and nufftct_umbrella_destroy serve both methods.
 *
 * Steps: F^-1, the inverse DFT of the N_phi x N_theta x N_r samples with the
 * 1/N_d that reproduces the samples, over the centred band m_d in
 * [-N_d/2, N_d/2); P, the Kaiser-Bessel scaling s_d(m_d) = 1/Psi(m_d/K_d)
 * (beta = 2.34 J) and zero padding to K_d = 2 N_d (the factor-2 oversampling
 * the section prefers for this kernel); F, the forward FFT of the K grid;
 * T_sparse, the J^3 Kaiser-Bessel taps at grid coordinate 2 t_d (t_d the
 * target's index coordinate), taps k0+1..k0+J with k0 = floor(2 t_d - J/2),
 * every axis wrapped mod K_d.  Every axis is treated as periodic, as the DFT
 * makes it: exact for phi, for rho where the Radon values vanish beyond the
 * object; targets in theta's unsampled polar caps get the periodic
 * interpolant's values (method 2 gives them zero taps).
 *
 * n_phi, n_theta, n_r: each even, in 8..512, with 2n = 2^a 3^b 5^c and among
 * the compiled lengths (8 12 16 20 24 30 32 36 40 48 60 64 72 80 90 96 120
 * 128 144 160 180 192 240 256 288 320 360 384 480 512); J in [2, 8].  Create
 * allocates the K_0 K_1 K_2 complex grid workspace on the current device
 * (8 x the radial data) and small tables; resample calls on one object
 * share that workspace, so calls that overlap race.  Errors: as method 2,
 * plus EUNSUPPORTED (length not compiled, weight fit) and ENOMEM.
 */
int nufftct_umbrella1_create(nufftct_umbrella** out, int64_t n_proj, int64_t n_alpha,
                             int64_t n_t, double source_radius, double source_detector,
                             double detector_side, int64_t n_phi, int64_t n_theta,
                             double theta0, double dtheta, int64_t n_r, int J, int precision,
                             void* stream);
/* Method 1 only: K3 (host, 3 values) receives the grid sizes (K_phi, K_theta, K_r). */
int nufftct_umbrella_grid_shape(const nufftct_umbrella* u, int64_t* K3);
/*
 * Method 1 only, one step at a time (device buffers, not aliasing):
 *   NUFFTCT_UMB_STAGE_GRID:   in = radial samples [phi][theta][rho] ->
 *                             out = F P F^-1 D on the K grid [K_phi][K_theta][K_r],
 *                             frequency kappa at index kappa mod K_d (out is
 *                             overwritten in full);
 *   NUFFTCT_UMB_STAGE_GATHER: in = such a grid -> out = umbrella samples [k][i][j].
 */
#define NUFFTCT_UMB_STAGE_GRID 0
#define NUFFTCT_UMB_STAGE_GATHER 1
int nufftct_umbrella_stage(nufftct_umbrella* u, int stage, const void* in, void* out,
                           void* stream);

/*
 * Umbrella derivative-Radon values -> cone-beam projections: the Grangeat
 * step in reverse (Section 2.2.2, Figures 2.14-2.15; its steps' costs in
 * eq 2.21-2.24), one projection per umbrella subset.  The section defers its
 * weights to an earlier report; they are taken from Grangeat's relation in
 * its textbook form.  Per projection k:
 *   1. de-postweighting: p'_ij = -U[k][i][j] R^2 / (R^2 + s'_j^2), the
 *      derivative of the 2D Radon transform of the pre-weighted projection on
 *      the virtual detector through the axis (s'_j = t_j R / D); the minus
 *      turns the umbrella orientation (normal (e x q)/|e x q|) into the one
 *      whose distance grows with s';
 *   2. radial FFTs of the lines zero-padded to 2n samples, times
 *      -i sign(k) / (2 pi) dalpha dk (inversion from derivative data needs no
 *      ramp); the k = 0 bin takes dalpha dk^2 / 6 P(alpha, 0) (the
 *      Euler-Maclaurin correction of the trapezoidal rule on |k| P at its
 *      kink, P(alpha, 0) = -int s' p' ds'); the Nyquist bin nothing;
 *   3. 2D NUFFT transpose: Kaiser-Bessel spreading (J taps per axis, beta =
 *      2.34 J, the neighbour rule of the projector) of the polar points
 *      omega = pi (m - n)/n (cos alpha_i, sin alpha_i) onto the 2n x 2n grid,
 *      the unnormalised inverse 2D FFT, the crop to n x n and 1/Psi per axis;
 *   4. de-preweighting: X = g sqrt(R^2 + u'^2 + v'^2) / R.
 * Geometry as the umbrella resampling (source radius R, source-detector
 * distance D, detector side, alpha_i = pi i / n_alpha, t_j = (j - n/2) side/n,
 * pixel (a, b) at u = (a - n/2) side/n, v = (b - n/2) side/n).  Projections
 * are exact (to the O(dk^4) quadrature error) where the object's shadow lies
 * inside the detector's inscribed disc: the umbrella lines reach |t| <= side/2.
 *
 * umbrella (device): n_proj * n_alpha * n complex, [k][i][j] (the umbrella
 * resampling's output with n_t = n).  out (device): n_proj * n * n complex,
 * [k][b][a] (v row, u column).  Complex64 for FP32, complex128 for FP64.
 * n: one of the compiled sizes 16 24 32 48 64 96 128 160 192 256 320 384
 * 512; J in [2, 8] (the paper's [5 5]: J = 5).  Create allocates on the current
 * device the spectra (n_alpha * 2n * n_proj complex), the row-pass workspace
 * (n_proj * 2n * n complex) and the per-cell gather lists of the polar points
 * (n_alpha * 2n * J^2 entries); calls on one object share them, so calls that
 * overlap race.  Errors: EINVAL (counts, distances, J, NULL or aliasing
 * buffers), EUNSUPPORTED (n not compiled), ENOMEM, EHIP.
 */
int nufftct_grangeat_create(nufftct_grangeat** out, int64_t n_proj, int64_t n_alpha, int64_t n,
                            double source_radius, double source_detector, double detector_side,
                            int J, int precision, void* stream);
int nufftct_grangeat_project(nufftct_grangeat* g, const void* umbrella, void* out, void* stream);
/*
 * One step at a time (device buffers, not aliasing):
 *   NUFFTCT_GR_STAGE_SPECTRA:     in = umbrella samples [k][i][j] -> out =
 *                                 filtered spectra c[(i * 2n + m) * n_proj + k]
 *                                 (steps 1-2; frequency (m - n) dk);
 *   NUFFTCT_GR_STAGE_BACKPROJECT: in = such spectra -> out = projections
 *                                 [k][b][a] (steps 3-4).
 * n_entries receives the number of gather-list entries (host pointer).
 */
#define NUFFTCT_GR_STAGE_SPECTRA 0
#define NUFFTCT_GR_STAGE_BACKPROJECT 1
int nufftct_grangeat_stage(nufftct_grangeat* g, int stage, const void* in, void* out,
                           void* stream);
int nufftct_grangeat_info(const nufftct_grangeat* g, int64_t* n_entries);
int nufftct_grangeat_destroy(nufftct_grangeat* g);

/*
 * Batch of independent volumes of uneven size (each with its own radial
 * direction set).  The batch owns one plan per volume (created with the
 * given parameters; J, kernel, beta and precision are shared), each with its
 * own workspace, so the volumes are independent.  With Kaiser-Bessel weights
 * and the radial stage, volumes of equal N, K and n_r on grids below 192^3
 * are grouped into units that run every stage as one launch across the
 * unit's volumes (FFT and radial passes over up to 64 volumes at once, the
 * point stages over all of them); larger volumes, and every volume of a
 * min-max batch, run their own plan's kernels.  The units are dealt to up
 * to four worker streams (longest-processing-time order by estimated cost)
 * that fork from the caller's stream and join back into it, so that units
 * run side by side.  Results equal the volumes' single plans bit for bit.
 * Arrays are HOST arrays of length nvol; dirs[b] is a HOST pointer to
 * n_lines[b] x 3 doubles.  Create also allocates the units' small device
 * tables.  Errors: EINVAL (a null array, nvol < 1, or any volume's plan
 * parameters, reported with its index), EUNSUPPORTED (a unit too large for
 * one launch per stage), ENOMEM, EHIP.
 */
int nufftct_batch_create(nufftct_batch** out, int nvol, const int64_t* N, const int64_t* K,
                         int J, int kernel, double beta, int precision,
                         const double* const* dirs, const int64_t* n_lines,
                         const int64_t* n_r, void* stream);

/*
 * As nufftct_batch_create, with each size class (volumes of equal N, K and
 * n_r) taking the tiling that nufftct_autotune_radial picks on the class
 * member with the most lines (which also records it for plans of that
 * geometry).  Tuning runs candidate plans on the GPU: seconds for large
 * classes.  Errors as nufftct_batch_create, plus EHIP from the tuner.
 */
int nufftct_batch_create_tuned(nufftct_batch** out, int nvol, const int64_t* N, const int64_t* K,
                               int J, int kernel, double beta, int precision,
                               const double* const* dirs, const int64_t* n_lines,
                               const int64_t* n_r, void* stream);

/* vols[b], outs[b]: device pointers per volume (sizes as for that volume's plan);
 * flags as for nufftct_forward / nufftct_adjoint (DETERMINISTIC included). */
int nufftct_batch_forward(nufftct_batch* batch, const void* const* vols, void* const* outs,
                          int flags, void* stream);
int nufftct_batch_adjoint(nufftct_batch* batch, const void* const* ins, void* const* vols,
                          int flags, void* stream);

/*
 * Capture the batch's forward (dir = 0) or adjoint (dir = 1) for fixed
 * buffers into a HIP graph owned by the batch (the worker streams become
 * parallel branches), and replay it with nufftct_batch_graph_launch.
 * Replays read and write the same buffers given here.  The stream must not
 * be NULL; stage timing is off inside the graph.
 */
int nufftct_batch_graph_capture(nufftct_batch* batch, int dir, const void* const* src,
                                void* const* dst, int flags, void* stream);
int nufftct_batch_graph_launch(nufftct_batch* batch, int dir, void* stream);

int nufftct_batch_destroy(nufftct_batch* batch);

/* Message for this thread's most recent failure ("" if none). */
const char* nufftct_last_error(void);

/* Library version string. */
const char* nufftct_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NUFFTCT_H */

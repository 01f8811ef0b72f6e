/*
 * dmwf.h -- C ABI of the dual messenger Wiener filter for CMB (I, Q, U) maps
 * on the sphere, for AMD MI355X (gfx950).
 *
 * Method: Kodi Ramanah, Lavaux & Wandelt (2018), "Optimal and fast E/B
 * separation with a dual messenger field".  The library solves the Wiener
 * filter equation (S^-1 + N^-1) s = N^-1 d (Sec. 1, eq 2) for joint
 * temperature and polarization data with the dual messenger iteration
 * (Sec. 2, eqs 8-9 and Algorithm 1), and produces constrained realizations
 * (Sec. 2.2, eq 19).  The paper's flat-sky FFT basis change (eqs 12-16) is
 * replaced by spin-0 + spin-2 spherical harmonic transforms on an
 * iso-latitude ring grid (HEALPix RING or Gauss-Legendre).
 *
 * Conventions shared by every call
 * --------------------------------
 * Maps      [nrhs][3][npix] doubles, fields (I, Q, U), pixels in RING order
 *           (rings from north to south, pixel j of a ring at
 *           phi = phi0 + 2 pi j / nphi).
 * alm       [nrhs][3][nalm][2] doubles, fields (T, E, B), interleaved
 *           complex (re, im), only m >= 0, packed m-major:
 *           idx(l, m) = m (2 lmax + 1 - m) / 2 + l, nalm = (lmax+1)(lmax+2)/2.
 *           Fields are real: a_{l,-m} = (-1)^m conj(a_lm).  E and B are zero
 *           for l < 2.
 * Harmonics Y_lm with the Condon-Shortley phase; spin-2 harmonics in the
 *           Goldberg et al. (1967) convention; polarization in the
 *           Zaldarriaga-Seljak (1997) convention:
 *           Q +- iU = sum_lm (+-2)a_lm (+-2)Y_lm, (+-2)a = -(a^E +- i a^B).
 * Transforms Y = alm2map (synthesis); Y^T = its plain adjoint (no weights,
 *           for sum_{l, m=-l..l} conj(a) b on coefficients and the real dot
 *           product on maps); A = Y^T W = map2alm with W the pixel
 *           quadrature weights (4 pi / npix on HEALPix).
 * Ownership The caller owns every buffer it passes.  Host-pointer calls copy
 *           inputs to the device and results back before returning.
 *           *_device calls borrow caller device buffers for the duration of
 *           the work they enqueue on the given HIP stream; NULL selects the
 *           plan's own stream (a stream the plan creates, not the null
 *           stream).  The single transforms (dm_alm2map_device,
 *           dm_map2alm_device) return once their work is enqueued; the
 *           Wiener filter calls return when it has finished (they read a
 *           non-finite count back from the device).  The plan owns all other
 *           device memory.
 * Threads   A plan is not thread-safe: use it from one host thread at a time.
 * Errors    Every call returns dm_status (0 = DM_OK).  On error nothing is
 *           written to outputs unless stated; dm_last_error() describes the
 *           last error on that plan.  No C++ exception crosses this ABI.
 */
#ifndef DMWF_H
#define DMWF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DMWF_ABI_VERSION 11

typedef enum {
    DM_OK = 0,
    DM_EINVAL = -1,        /* invalid argument or input data            */
    DM_ENOMEM = -2,        /* device or host allocation failed          */
    DM_EDEVICE = -3,       /* no usable GPU, or a HIP runtime error     */
    DM_ENONFINITE = -4,    /* a non-finite value appeared in the iterate */
    DM_ESTATE = -5,        /* call out of order (e.g. no noise set yet)  */
    DM_EUNSUPPORTED = -6   /* valid request that the library cannot run */
} dm_status;

typedef enum { DM_GRID_HEALPIX_RING = 0, DM_GRID_GAUSS_LEGENDRE = 1 } dm_grid_kind;

/* DM_FP64: every step in double precision.
 * DM_MIXED: Legendre recursion, seeds and rescaling in double precision;
 *           harmonic-coefficient contraction and the ring-Fourier data in
 *           single precision; the iterate alm and the final residual in
 *           double precision.  I/O buffers are always double.            */
typedef enum { DM_FP64 = 0, DM_MIXED = 1 } dm_precision;

/* Per-pixel noise covariance layout (eq 11).
 * DM_NCOV_DIAG3: [3][npix] variances (II, QQ, UU), N_p diagonal.
 * DM_NCOV_SYM6:  [6][npix] the symmetric 3x3 block of eq 11 in the order
 *                (II, IQ, IU, QQ, QU, UU): correlated noise.              */
typedef enum { DM_NCOV_DIAG3 = 0, DM_NCOV_SYM6 = 1 } dm_ncov;

typedef struct {
    int kind;      /* dm_grid_kind                                        */
    int nside;     /* HEALPix resolution (kind 0)                         */
    int ntheta;    /* Gauss-Legendre rings (kind 1)                       */
    int nphi;      /* pixels per Gauss-Legendre ring (kind 1)             */
} dm_grid;

/* Cooling schedule (Algorithm 1, Sec. 3.2), xi = lambda * tau, in one of
 * two modes.
 *
 * Fixed mode (iters_per_step >= 1): lambda_k = lambda_start^(1 - k/(nsteps-1)),
 * k = 0..nsteps-1 (the last step has lambda = 1, i.e. mu = 0), with
 * iters_per_step iterations per step; nsteps = 1 runs only lambda = 1.
 *
 * Epsilon mode (iters_per_step <= 0): Algorithm 1's own loop.  lambda_j =
 * lambda_start * beta^j while above 1, then a last step at lambda = 1; at
 * step j the iteration repeats until the Cauchy ratio
 * ||u_i - u_{i-1}|| / ||u_i|| (harmonic L2 over T, E, B with m > 0 counted
 * twice; u_0 = 0; the largest over the right-hand sides of a batch) falls
 * below eps_j = max(eps_end, eps_start * eps_eta^-j), and below eps_end at
 * the last step (the threshold cooling of Sec. 3.2); the solve stops early
 * after max_iters iterations in total.  nsteps is ignored.
 *
 * In both modes max_iters > 0 stops a solve once that many iterations
 * have run in total, counted from the start of the schedule (a resumed
 * solve counts the iterations before its checkpoint); the solve returns
 * the iterate reached, and dm_checkpoint_save can record it.  Fixed mode
 * accepts max_iters = 0 (no cap).                                        */
typedef struct {
    double lambda_start;   /* >= 1                                          */
    int nsteps;            /* fixed mode: >= 1                              */
    int iters_per_step;    /* fixed mode: >= 1; <= 0 selects epsilon mode   */
    double beta;           /* epsilon mode: cooling factor, 0 < beta < 1    */
    double eps_start;      /* epsilon mode: first threshold, >= eps_end     */
    double eps_end;        /* epsilon mode: final threshold, > 0            */
    double eps_eta;        /* epsilon mode: relaxation per step, >= 1       */
    int max_iters;         /* cap on the total: >= 1 (epsilon), >= 0 (fixed)*/
} dm_schedule;

/* Per right-hand side diagnostics.  residual = ||A x - y|| / ||y|| with
 * A = 1 + S^1/2 Y^T N^-1 Y S^1/2, x = S^+1/2 u, y = S^1/2 Y^T N^-1 d
 * (Appendix C); chi2 = (d - Y u)^T N^-1 (d - Y u) + u^T S^+ u (eq 3);
 * cauchy = ||u_i - u_{i-1}|| / ||u_i|| at the last iteration (Algorithm 1's
 * stopping ratio); seconds = wall time of the whole call.               */
typedef struct {
    int iterations;
    double residual;
    double cauchy;
    double chi2;
    double seconds;
} dm_stats;

typedef struct dm_plan dm_plan;   /* opaque; owns all device memory */

/* ABI version of the loaded library (DMWF_ABI_VERSION).                   */
int dm_abi_version(void);

/* Number of visible HIP devices (0 when there is none).                   */
int dm_device_count(void);

/* Create a plan for a grid, band limit lmax (>= 2, and <= 3 nside - 1 on
 * HEALPix, <= ntheta - 1 and <= (nphi - 1) / 2 on Gauss-Legendre), up to
 * max_rhs right-hand sides per call, on HIP device `device`.  Builds ring
 * tables, recursion coefficients and the per-(m, ring) recursion seeds.
 * Returns DM_EDEVICE without a GPU, DM_EINVAL on bad sizes,
 * DM_EUNSUPPORTED for a ring length that the library's FFT cannot stage.
 *
 * Environment variables read here, for tuning and testing; none changes a
 * result beyond FP rounding except DMWF_RING_FP32:
 *   DMWF_MFMA=0|1          batched matrix-core Legendre kernels off / on
 *   DMWF_SYN_MCHUNK, DMWF_ANA_MCHUNK   their m-chunk per XCD (see dm_autotune)
 *   DMWF_SYN_WAVES=1|2|4|8 waves per block of the batched synthesis
 *   DMWF_RING_BIG_THREADS, DMWF_RING_SMALL_THREADS   ring size-class widths
 *   DMWF_SYN_THREADS, DMWF_SYN_R, DMWF_ANA_R   single-RHS kernel tiling
 *   DMWF_GRAPHS=0          fixed-schedule steps launched directly, not as graphs
 *   DMWF_RING_THREADS=256|512|1024     whole-ring workgroup width
 *   DMWF_RING_CLASSES=0    unsplit rings in one launch, not two by size
 *   DMWF_RING_SMALL_M=n    size bound of the two launches (tests)
 *   DMWF_FFT_MAX_ELEMS=n   largest unsplit transform buffer (tests: split rings)
 *   DMWF_FUSE6=0           3x3 noise update as a pass of its own
 *   DMWF_RING_FP32=1       FP32 ring transforms on DM_MIXED plans (lower
 *                          accuracy: about 1.2e-5 at Nside 1024, past 1e-5)
 *   DMWF_TUNE_CACHE=path   dm_autotune's cache file                       */
dm_status dm_plan_create(dm_plan** plan, const dm_grid* grid, int lmax, int max_rhs,
                         dm_precision precision, int device);
dm_status dm_plan_destroy(dm_plan* plan);

/* Grid facts of a plan: npix, nalm, number of rings.                       */
dm_status dm_plan_info(const dm_plan* plan, int64_t* npix, int64_t* nalm, int* nrings);

/* Signal covariance (eq 10): cl [4][lmax+1] in the order TT, EE, BB, TE.
 * Each S_l must be positive semi-definite (TE^2 <= TT EE, all >= 0) and
 * finite; E and B entries below l = 2 are ignored.                        */
dm_status dm_set_spectra(dm_plan* plan, const double* cl);

/* Noise covariance (eq 11) with one mask common to I, Q and U:
 * dm_set_noise_masks(plan, ncov, layout, obs, obs).                       */
dm_status dm_set_noise(dm_plan* plan, const double* ncov, dm_ncov layout, const uint8_t* obs);

/* Noise covariance (eq 11) with distinct temperature and polarization masks
 * (Appendix B).  ncov: host [3][npix] (DM_NCOV_DIAG3) or [6][npix]
 * (DM_NCOV_SYM6), copied.  obs_t: host [npix], nonzero = I observed;
 * obs_p: host [npix], nonzero = Q and U observed; NULL = all observed.
 *
 * The inverse noise covariance P_p is the block of N_p^-1 on the observed
 * components with zero rows and columns elsewhere: Appendix B's
 * N = Sigma C Sigma with Sigma^-1 = 0 on unobserved components (for
 * diagonal noise, 1 / variance on observed components).  The messenger
 * covariance of eq 4 is T_p = tau / w_p with w_p the pixel weight and
 * tau = min over pixels with an observed component of w_p / lambda_max(P_p)
 * (the smallest eigenvalue of N_p times w_p when all is observed); the
 * update of eq 9 is t = (1 - T_p P_p) u_x + T_p P_p d.
 *
 * Requirements (else DM_EINVAL, nothing changed): DM_NCOV_DIAG3 - every
 * observed component's variance finite and > 0; DM_NCOV_SYM6 - on every
 * pixel with an observed component all six entries finite and N_p
 * positive definite (its unobserved components enter through the
 * correlation matrix C); at least one observed component.  Entries of
 * pixels with nothing observed are ignored.  Another layout value is
 * DM_EUNSUPPORTED.  With DM_NCOV_SYM6 the three fields of a pixel are
 * coupled, so an iteration cannot keep one field's ring in fast memory from
 * synthesis to analysis: it writes u_x = Y u and forms t from the three
 * fields as the next ring analysis loads them, which costs a little more
 * than diagonal noise (DMWF_FUSE6=0 runs the update as a pass of its own). */
dm_status dm_set_noise_masks(dm_plan* plan, const double* ncov, dm_ncov layout, const uint8_t* obs_t,
                             const uint8_t* obs_p);

/* Cooling schedule; the default is the fixed mode {1e3, 20, 10}.          */
dm_status dm_set_schedule(dm_plan* plan, const dm_schedule* schedule);

/* Per-iteration record of the last solve in epsilon mode (Fig. 4's Cauchy
 * trace): cauchy[i] = the Cauchy ratio after iteration i (largest over the
 * right-hand sides), step[i] = its cooling step.  Copies min(cap, n)
 * entries into the caller's host arrays (either may be NULL) and sets *n to
 * the iteration count; *n = 0 after a fixed-mode solve.  Errors: DM_EINVAL
 * for a null plan or n.                                                    */
dm_status dm_schedule_trace(const dm_plan* plan, double* cauchy, int* step, int cap, int* n);

/* Adaptive working resolution (the hierarchical framework of the text
 * after eq 9 and the working-resolution proposal of Sec. 4).  At cooling
 * step k, with mu_k = (lambda_k - 1) tau, the prior clamped at mu_k is mu_k 1
 * in T, E and B above ell_iter(mu_k), the largest l whose S_l (the TE block
 * and BB) has an eigenvalue >= mu_k; the step then runs its harmonic update
 * with the band limit L_k = min(lmax, max(2, ceil(factor ell_iter(mu_k)))):
 * u = P_L F t_hat, coefficients above L_k set to zero, and the transforms
 * skip the degrees and orders above L_k.  The pixel grid, K and b stay those
 * of the data.  The last step (mu = 0) always runs the full band.  factor
 * 0 (the default) turns it off, factor >= 1 turns it on for later Wiener
 * filter solves (not dm_iterate); other values are DM_EINVAL.            */
dm_status dm_set_adaptive_resolution(dm_plan* plan, double factor);

/* Band limit L_k of each cooling step of the last solve's schedule (lmax
 * for every step when adaptive resolution is off).  Copies min(cap, n)
 * values to the caller's host array (NULL allowed), sets *n to the number
 * of cooling steps.  Errors: DM_EINVAL for a null plan or n.              */
dm_status dm_step_band_limits(const dm_plan* plan, int* lcut, int cap, int* n);

/* Diagnostics trace (Fig. 4's chi^2 and residual panels): with every > 0,
 * every later Wiener filter solve evaluates, for the iterate u_i after
 * iteration i (counted from the start of the schedule), the chi^2 of eq 3
 * and the Appendix C residual, both as dm_stats defines them, whenever i is
 * a multiple of `every` and after the solve's last iteration.  Each record
 * costs one FP64 synthesis and one FP64 adjoint transform, and a traced
 * solve launches its kernels directly (no graphs); the iterates themselves
 * are unchanged.  Corrections of the refinement are not traced.  every = 0
 * (the default) turns it off; every < 0 is DM_EINVAL.                      */
dm_status dm_set_diagnostics(dm_plan* plan, int every);

/* The trace of the last solve: iteration[k], and chi2[k * nrhs + r],
 * residual[k * nrhs + r] for right-hand side r.  Copies min(cap, n)
 * entries (times nrhs values) into the caller's host arrays (each may be
 * NULL), sets *n to the entry count and *nrhs (nullable) to that solve's
 * nrhs; both 0 when the last solve was not traced.  Errors: DM_EINVAL for a
 * null plan or n.                                                         */
dm_status dm_diagnostics_trace(const dm_plan* plan, int* iteration, double* chi2, double* residual, int cap, int* n,
                               int* nrhs);

/* Refinement by Appendix A's modified Jacobi relaxation: every later
 * Wiener filter solve (also inside dm_constrained_realizations) follows
 * its messenger run with ncorrections corrections
 *     s <- s + W~(g),  g = W Y r,  r = Pi Y^T P (d - Y s) - S^+ s,
 * r the residual of the Wiener filter equation on the range of S (eq 2;
 * Pi the projector onto it, S^+ the pseudo-inverse, P as for
 * dm_set_noise_masks), evaluated with FP64 transforms in either precision,
 * and W~ the same fixed-schedule messenger run driven by the weighted
 * data g (b = T_p g) from t = 0.  W Y, the pixel weights times synthesis,
 * is a right inverse of the adjoint Y^T where the quadrature is exact; it
 * takes the place of the paper's flat-sky d - W^+ s (eq A1), and the fixed
 * point solves the Wiener filter equation exactly on any grid on which
 * Y^T W Y is invertible, so the corrections also remove the messenger's
 * own HEALPix quadrature bias and, on a DM_MIXED plan, the FP32 rounding.
 * Each correction costs one messenger run plus three FP64 transforms.  The
 * corrections converge only where W~ approximates the inverse well enough
 * (on Gauss-Legendre grids; on HEALPix with a moderate noise range and
 * mask); elsewhere they stall or grow, which dm_refinement_trace shows.
 * A refined solve returns the last iterate, as Appendix A's relaxation
 * does; dm_set_refinement_select can ask for the iterate of smallest
 * residual norm instead.
 * ncorrections in [0, 1000], 0 = off (the default), else DM_EINVAL;
 * allocates a map and an alm buffer for max_rhs right-hand sides when
 * first enabled (DM_ENOMEM).  In epsilon mode the first solve runs under
 * the Cauchy rule and every correction runs the iterations it spent at
 * each cooling step (Appendix A's prescription; dm_schedule_trace keeps the
 * first solve's record).  A refined solve needs no iteration cap on the
 * fixed schedule and no pending checkpoint (else DM_EUNSUPPORTED from the
 * solve), leaves nothing for
 * dm_checkpoint_save, and reports in dm_stats the iterations of all runs
 * and `cauchy` = 0 (the residual history is the convergence record).      */
dm_status dm_set_refinement(dm_plan* plan, int ncorrections);

/* Which iterate a refined solve returns: keep_best = 0 (the default) the
 * last one, Appendix A's result; keep_best = 1, per right-hand side, the
 * iterate of smallest ||r|| / ||Pi Y^T P d|| among the plain solve and the
 * corrections (the first of equal ones), which is never worse than the
 * plain solve where the corrections diverge.  Other values: DM_EINVAL.    */
dm_status dm_set_refinement_select(dm_plan* plan, int keep_best);

/* For the last refined solve, index[r] = the k of the iterate right-hand
 * side r returned (k = 0 the plain solve, k = ncorrections the last
 * correction; it indexes dm_refinement_trace's history).  Copies
 * min(cap, n) entries to the caller's host array (NULL allowed) and sets
 * *n to that solve's nrhs, 0 before any refined solve.  Errors: DM_EINVAL
 * for a null plan or n.                                                   */
dm_status dm_refinement_selected(const dm_plan* plan, int* index, int cap, int* n);

/* Residual history of the last refined solve: history[k * nrhs + r] =
 * ||r_k|| / ||Pi Y^T P d|| for right-hand side r before correction k
 * (k = 0 .. ncorrections - 1) and after the last (k = ncorrections), the
 * norms harmonic L2 with m > 0 counted twice.  Copies min(cap, n) values
 * to the caller's host array (NULL allowed), sets *n = (ncorrections + 1)
 * nrhs and *nrhs (NULL allowed) to that solve's nrhs; both 0 before any
 * refined solve.  Errors: DM_EINVAL for a null plan or n.                 */
dm_status dm_refinement_trace(const dm_plan* plan, double* history, int cap, int* n, int* nrhs);

/* Wiener filter of nrhs data maps d [nrhs][3][npix] (Algorithm 1).  Writes
 * the final iterate u (the Wiener-filtered T, E, B alm) to alm
 * [nrhs][3][nalm][2], optionally the map Y u to map [nrhs][3][npix]
 * (nullable), and optionally diagnostics to stats[nrhs] (nullable; the
 * residual and chi2 cost two extra adjoint transforms).  Masked pixels of
 * d are ignored.  DM_ENONFINITE if the iterate became non-finite.        */
dm_status dm_wiener_filter(dm_plan* plan, int nrhs, const double* d, double* alm, double* map,
                           dm_stats* stats);

/* Same on device buffers (double): d, alm, map (nullable) are device
 * pointers; work is enqueued on hip_stream.  stats (host, nullable) forces
 * a synchronisation at the end.                                          */
dm_status dm_wiener_filter_device(dm_plan* plan, int nrhs, const void* d, void* alm, void* map,
                                  void* hip_stream, dm_stats* stats);

/* Same with single-precision device I/O (float d [nrhs][3][npix], alm
 * [nrhs][3][nalm][2], map nullable), for callers that keep FP32 maps, e.g.
 * with a DM_MIXED plan: the inputs are widened to double on the device, the
 * solve is the double-buffer one, and alm and map are rounded to float, so
 * the results are those of dm_wiener_filter_device on the widened data,
 * rounded.  Allocates device scratch for the double buffers (DM_ENOMEM);
 * non-finite data are DM_EINVAL.                                          */
dm_status dm_wiener_filter_device_f32(dm_plan* plan, int nrhs, const void* d, void* alm, void* map,
                                      void* hip_stream, dm_stats* stats);

/* Constrained realizations, eq 19: s_CR,k = W(d - d_hat_k) + s_hat_k for
 * k < nreal, run as one batch of nreal + 1 right-hand sides (the extra one
 * is W d).  d [3][npix]; shat_alm [nreal][3][nalm][2]; dhat
 * [nreal][3][npix] (fake data Y s_hat + n_hat made by the caller);
 * scr_alm [nreal][3][nalm][2]; f_alm (nullable) receives the fluctuation
 * parts f_k = s_CR,k - W d.  Needs max_rhs >= nreal + 1.                 */
dm_status dm_constrained_realizations(dm_plan* plan, int nreal, const double* d,
                                      const double* shat_alm, const double* dhat,
                                      double* scr_alm, double* f_alm);

/* Single transforms (host buffers), nrhs at a time.                       */
dm_status dm_alm2map(dm_plan* plan, int nrhs, const double* alm, double* map);          /* Y     */
dm_status dm_map2alm(dm_plan* plan, int nrhs, const double* map, double* alm);          /* Y^T W */
dm_status dm_alm2map_adjoint(dm_plan* plan, int nrhs, const double* map, double* alm);  /* Y^T   */

/* Single transforms on device buffers (double), enqueued on hip_stream.   */
dm_status dm_alm2map_device(dm_plan* plan, int nrhs, const void* alm, void* map, void* hip_stream);
dm_status dm_map2alm_device(dm_plan* plan, int nrhs, const void* map, void* alm, void* hip_stream);

/* dm_map2alm_device without any device allocation, for callers that
 * cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the ring Fourier data and the
 * partial-sum slots of the analysis live in a fixed array of 32 MiB that
 * the library's code object holds on every GPU it runs on (until the
 * process ends), not in the plan's buffers.  Same arguments, layouts and
 * results as dm_map2alm_device (the same kernels in the same order, so the
 * same values to the last bit); map and alm are caller device buffers, work
 * is enqueued on hip_stream (NULL = the plan's stream) and the call returns
 * once it is enqueued.  The call does not wait for earlier work of the plan
 * on other streams, and every call on one GPU shares its array, which keeps
 * the last call's contents: calls that overlap on one GPU race.  A call
 * whose work memory (ring data plus partial sums, for nrhs right-hand
 * sides) exceeds 32 MiB is refused with DM_EINVAL and a message giving the
 * size; DM_EDEVICE if the array's device address could not be obtained
 * when the plan was created.  Per-kernel timing is off during the call.    */
dm_status dm_map2alm_device_noalloc(dm_plan* plan, int nrhs, const void* map, void* alm, void* hip_stream);

/* Run `niter` messenger iterations at a fixed lambda (mu = (lambda-1) tau)
 * from a given messenger map t_in [nrhs][3][npix] (no masking applied to
 * it), with the data d [nrhs][3][npix] of the current noise setup:
 *   t_hat = A t, u = F^mu t_hat, u_x = Y u, t = K u_x + b.
 * Writes the last u to alm and the last t to t_out (nullable).  Used to
 * check single iterations step by step.                                  */
dm_status dm_iterate(dm_plan* plan, int nrhs, const double* d, const double* t_in, double lambda,
                     int niter, double* alm, double* t_out);

/* Checkpoint and resume of a Wiener filter solve.
 *
 * dm_checkpoint_save writes the state where the plan's last
 * dm_wiener_filter / dm_wiener_filter_device call stopped (normally at the
 * end of the schedule, earlier under a max_iters cap) to the file path:
 * the iterate u of every RHS (and the one before it in fixed mode), the
 * iterations done, the cooling step reached, the epsilon-mode trace, the
 * schedule, and fingerprints of the spectra, the noise and mask, and the
 * masked data.  The file (versioned, with a checksum) is written to
 * path + ".tmp" and renamed.  DM_ESTATE if no such solve has completed on
 * this plan; DM_EINVAL if the file cannot be written.
 *
 * dm_checkpoint_load reads such a file into the plan (same grid, lmax and
 * precision, nrhs <= max_rhs, else DM_EINVAL; a damaged or truncated file
 * is DM_EINVAL).  The next Wiener filter call then continues from it
 * instead of starting afresh: it must pass the same nrhs and data, with the
 * same spectra, noise and mask set and the same schedule except max_iters
 * (else DM_EINVAL, and the checkpoint stays loaded).  It runs the remaining
 * iterations (up to the current max_iters) and returns exactly, to the last
 * bit, what one uninterrupted call would have returned.  The constrained
 * realization call neither uses nor changes the checkpoint state.       */
dm_status dm_checkpoint_save(const dm_plan* plan, const char* path);
dm_status dm_checkpoint_load(dm_plan* plan, const char* path);

/* Autotuner of the launch shapes of a solve with nrhs right-hand sides,
 * timed on the plan's own buffers, keeping the fastest for this plan:
 *  - batched matrix-core Legendre kernels (from 2 RHS on for DM_MIXED, 8
 *    for DM_FP64): the synthesis' waves per block (1, 2, 4, 8) together with
 *    its m-chunk, and the analysis' m-chunk (how many consecutive m a chunk
 *    of workgroups on one XCD covers: 0, 1, 2, 4, 8).  These only move work
 *    between waves, workgroups and XCDs: results stay the same to the last
 *    bit;
 *  - the ring step's two launches by transform size (from 4 RHS on, where
 *    the plan has both size classes): workgroup widths of the large (512,
 *    1024) and the small transforms (256, 512, 1024).  A width changes the
 *    order of a few first-pixel rotation products: results move by FP64
 *    rounding only.
 * choice (nullable, [5]) receives the synthesis m-chunk, the analysis
 * m-chunk, the synthesis waves, the large and the small ring widths; ms
 * (nullable, [3]) the best synthesis, analysis and ring-step times per
 * launch (0 for a part not tuned or when the choice came from the cache).
 * With the environment variable DMWF_TUNE_CACHE naming a file, choices are
 * looked up there first (key: grid, lmax, precision, column tiles of 8 RHS,
 * ring classes) and new ones appended.  Leaves the plan unchanged (DM_OK,
 * choice = current values, ms = 0) when nrhs uses neither.  Call between
 * solves; it overwrites the plan's transform work buffers.               */
dm_status dm_autotune(dm_plan* plan, int nrhs, int* choice, double* ms);

/* Work of one Legendre transform of this plan, per right-hand side:
 * *points = ring pairs x nalm, the (l, m, ring pair) points of the
 * separable transform, and *executed = the points at or above each
 * (m, ring pair)'s start degree (below it the associated Legendre functions
 * are under 2^-100 of their scale and the recursion and contraction skip
 * them; the seeds fix it when the plan is made).  Errors: DM_EINVAL for a
 * null argument.                                                          */
dm_status dm_transform_work(dm_plan* plan, int64_t* points, int64_t* executed);

/* Per-kernel GPU timing, measured with HIP events on the plan's stream
 * when enabled: enable != 0 turns recording on and clears the totals.
 * dm_kernel_times writes, for kernel class k < *count (0 Legendre
 * analysis, 1 Legendre synthesis, 2 ring FFT + pointwise, 3 combine and
 * filter, 4 the separate 3x3 pixel update), the total milliseconds to ms[k] and the number of launches to
 * launches[k].                                                            */
dm_status dm_profile_enable(dm_plan* plan, int enable);
dm_status dm_kernel_times(dm_plan* plan, double* ms, int64_t* launches, int* count);

/* Text of the last error on this plan (or of the last failed
 * dm_plan_create when plan is NULL).  Valid until the next call.          */
const char* dm_last_error(const dm_plan* plan);

#ifdef __cplusplus
}
#endif

#endif /* DMWF_H */

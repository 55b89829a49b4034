/*
 * tfs.h -- C ABI of the MI355X time-fractional extra-stress update.
 *
 * The library advances, independently at every point of a grid, the
 * kernel-compressed time-fractional macroscopic Fokker-Planck system of a dilute
 * Hookean polymer solution under a prescribed velocity gradient kappa = grad u
 * (homogeneous flow: no advection, no centre-of-mass diffusion).  In tensor
 * variables X = C - I (conformation minus identity, symmetric) the model is
 *
 *   dX/dt = A_kappa(D^{1-alpha} X) + S_kappa D^{1-alpha} 1,      tau = gamma D^{1-alpha} X,
 *   A_kappa(Y) = kappa Y + Y kappa^T - Y/De,   S_kappa = kappa + kappa^T,   gamma = eta_p/De,
 *
 * i.e. the tested configuration operator of Sec. 3.2 (eq. conf_op_tested) with
 * a = 1/sqrt(2), the Riemann-Liouville derivative of Sec. 1 placed on the right-hand
 * side, and Kramers' stress for a unit-mass density.  The memory kernel
 * t^(alpha-1)/Gamma(alpha) is replaced by sum_k w_k exp(-lambda_k t) (Sec. 2.2), each
 * exponential carried as a fractional-mode field X_k, and time is discretised by the
 * BDF2 scheme of Sec. 4.1 (eqs. BDF_Phi_k_n+1 and FP_discrete) after one SDIRK2 step.
 *
 * Every function is extern "C", never throws, and returns a tfs_status.  Device
 * pointers are HIP device addresses; "host" pointers are ordinary memory.
 *
 * Packed symmetric components (c = d(d+1)/2):  2-D (xx, yy, xy);  3-D (xx, yy, zz, xy, xz, yz).
 * Velocity gradient components (d*d):          row-major kappa_ij = d u_i / d x_j.
 * Every field is structure-of-arrays with the point index fastest and a plane
 * stride of `stride` elements (>= npoints) between consecutive planes.  The
 * fractional-mode ring may instead be tiled: with tile T > 0 the points are cut into
 * tiles of T consecutive points and mode (slot, k, s) of point p lives at element
 *     ((slot * (stride/T) + p/T) * m * c + k * c + s) * T + p % T,
 * so all modes of a tile are contiguous (T = 0 is the plain [2][m][c][stride] layout).
 * Tiling keeps the number of concurrently streamed DRAM regions small.
 */
#ifndef TFS_H
#define TFS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TFS_OK = 0,
    TFS_EINVAL = 1,       /* invalid argument (message from tfs_last_error) */
    TFS_ENOMEM = 2,       /* device or host allocation failed (plan creation only) */
    TFS_EHIP = 3,         /* a HIP runtime call failed */
    TFS_ENUMERIC = 4,     /* TFS_FLAG_CHECK_SYNC: a non-finite value or a non-positive-definite C appeared */
    TFS_EUNSUPPORTED = 5  /* valid request this build does not implement */
} tfs_status;

typedef enum {
    TFS_FP64 = 0,         /* modes stored and updated in FP64 */
    TFS_FP32_MODES = 1    /* modes stored in FP32; recombination, solve, X, tau and all coefficients in FP64 */
} tfs_precision;

/*
 * Time discretisation of the modes and the state.
 *
 * TFS_SCHEME_BDF2 -- the paper's scheme (Sec. 4.1): BDF2 for the state and the modes,
 *   one SDIRK2 start-up step; two mode levels (a two-slot ring).
 * TFS_SCHEME_EXP -- an extension, not the paper's scheme: each mode solves its equation
 *   X_k' = -lambda_k X_k + w_k X (Sec. 2.2) exactly over a step on which X is linear in
 *   time, X_k^{n+1} = e_k X_k^n + w_k dt (a0_k X^n + a1_k X^{n+1}) with z = lambda_k dt,
 *   e_k = exp(-z), a0_k = (1 - (1+z) e_k)/z^2, a1_k = (z - 1 + e_k)/z^2; and since
 *   D^{1-alpha} X = sum_k X_k', the state equation is integrated over the step as
 *   X^{n+1} - X^n = A_kappa~(sum_k (X_k^{n+1} - X_k^n)) + S_kappa~ sum_k (mu_k^{n+1} - mu_k^n)
 *   (mu_k the modes of the constant 1), exact for a constant kappa, with kappa~ at the
 *   half step.  One step, one mode level updated in place: two mode accesses per
 *   mode-component and step instead of three, half the mode memory.
 */
typedef enum {
    TFS_SCHEME_BDF2 = 0,
    TFS_SCHEME_EXP = 1
} tfs_scheme;

/*
 * Storage precision of the velocity-gradient fields kappa_a, kappa_b a plan's steps read.
 * The extrapolation kappa~ = 2 kappa^n - kappa^{n-1} (eq. BDF_and_extrapolation) and all
 * arithmetic with it are FP64 either way; FP32 storage halves the gradient's share of the
 * memory traffic of the FP32-mode form.  Gradient adjoints (kappabar) stay FP64.
 */
typedef enum {
    TFS_KAPPA_FP64 = 0,
    TFS_KAPPA_FP32 = 1    /* FP32-mode plans only; no spatial form, coupled or transport step */
} tfs_kappa_precision;

/*
 * How a TFS_SCHEME_BDF2 plan stores its fractional modes (the arithmetic of the scheme is the
 * same; only what is stored, and so what FP32 storage rounds, differs):
 *   TFS_MODE_FORM_Y  Y_k^j = X_k^j - c_k X^j.  The new level Y_k^{n+1} = d_k h_k + d_k c_k P is
 *                    known before the local solve, so the modes stream once.  X ring: 2 slots.
 *   TFS_MODE_FORM_Z  Z_k^j = Y_k^j - beta_k X^{j-1} with beta_k = w_k/lambda_k - c_k for the
 *                    modes that relax within the plan's horizon (lambda_k max_steps dt >= 1),
 *                    beta_k = 0 for the others (lambda_k = 0 included), and X^{-1} = 0: the
 *                    quasi-static part (w_k/lambda_k) X of a mode that follows X is taken out,
 *                    so the stored value is small.  Its
 *                    new level Y_k^{n+1} - beta_k X^n is still known before the solve; reading
 *                    level n-1 back needs X^{n-2}, so the X ring holds 3 levels.  The stress is a
 *                    near-cancelling sum over the modes: with FP32 storage this form rounds it
 *                    about ten times less (measured at alpha = 0.2, m = 48, 2000 steps).
 *   TFS_MODE_FORM_AUTO  Z for FP32-mode BDF2 plans, Y otherwise.
 * TFS_SCHEME_EXP plans have their own one-level form (tfs_scheme).
 */
typedef enum {
    TFS_MODE_FORM_AUTO = 0,
    TFS_MODE_FORM_Y = 1,
    TFS_MODE_FORM_Z = 2
} tfs_mode_form;

enum {
    TFS_FLAG_CHECK_SYNC = 1u << 0  /* tfs_step synchronises and returns TFS_ENUMERIC on non-finite/non-PD diagnostics */
};

typedef struct tfs_plan_s* tfs_plan;

typedef struct {
    int32_t dim;          /* 2 or 3 */
    int32_t nmodes;       /* 1 <= m <= 256 exponential modes */
    int64_t npoints;      /* points updated by each call (>= 0) */
    int64_t stride;       /* plane stride in elements; 0 means npoints rounded up to a multiple of tile;
                             must be >= npoints and, with tile > 0, a multiple of tile */
    int64_t tile;         /* mode-ring tile in points: 0 (untiled) or a positive multiple of 4; with
                             more than one tile, (tile + 256) * m * c * 8 must stay below 2^31 */
    double alpha;         /* fractional order in (0, 1]; kept for reporting and gradients */
    double De;            /* relaxation time (Deborah/Weissenberg number) > 0 */
    double eta_p;         /* polymer viscosity (1-beta)/Re >= 0; gamma = eta_p/De (Sec. 1, Kramers) */
    double dt;            /* time step > 0 */
    int64_t max_steps;    /* time levels 0..max_steps may be produced; tfs_step accepts n < max_steps */
    const double* w;      /* host [m] weights w_k >= 0, finite (copied) */
    const double* lambda; /* host [m] poles lambda_k >= 0, finite (copied) */
    int32_t precision;    /* tfs_precision */
    uint32_t flags;       /* TFS_FLAG_* */
    void* stream;         /* hipStream_t the plan launches on (NULL = default stream) */
    int32_t scheme;       /* tfs_scheme */
    int32_t kappa_precision;  /* tfs_kappa_precision (0 = FP64) */
    int32_t mode_form;        /* tfs_mode_form (0 = AUTO) */
} tfs_plan_desc;

/*
 * Create a plan: validates the descriptor, copies (w, lambda), and precomputes in
 * FP64 on the host the per-mode BDF2 factors of Sec. 4.1 (d_k = 1/(b0 + lambda_k dt),
 * c_k = w_k dt d_k, eta_k = lambda_k dt d_k, eta = sum_k b0 c_k, b = (3/2, -2, 1/2)),
 * the SDIRK2 start-up factors, and the table zeta^n of the spatially uniform mass
 * mode's memory term (the mass mode Phi_000 = 1 of Sec. 3.4 and its fractional modes
 * are the same at every point, so its contribution is one scalar per step).  These
 * tables are uploaded once.  The plan owns them and a small reduction buffer.
 * Errors: TFS_EINVAL (dim not 2/3, m < 1, npoints < 0, stride < npoints, alpha not in
 * (0,1], De <= 0, eta_p < 0, dt <= 0, max_steps < 1, null or negative/non-finite w or
 * lambda, unknown precision or scheme, tile negative or not a multiple of 4, stride not
 * a multiple of a positive tile, an unknown kappa precision or FP32 velocity gradients with
 * FP64 modes, an unknown mode form or TFS_MODE_FORM_Z with TFS_SCHEME_EXP), TFS_ENOMEM,
 * TFS_EHIP.  *out is NULL on error.
 * With TFS_SCHEME_EXP the per-mode factors are e_k, a0_k and a1_k of tfs_scheme and the
 * mass-mode table holds the increments sum_k (mu_k^{n+1} - mu_k^n).
 */
tfs_status tfs_plan_create(const tfs_plan_desc* desc, tfs_plan* out);

/* Release a plan (NULL is accepted).  Synchronises its stream first. */
tfs_status tfs_plan_destroy(tfs_plan plan);

/* Rebind the stream later launches use. */
tfs_status tfs_plan_set_stream(tfs_plan plan, void* stream);

/*
 * Spatial form: centre-of-mass diffusion eps Laplace on a periodic grid with u = 0
 * (Sec. 4.1, eq. FP_discrete with L = -eps Laplace - A(kappa~)), solved where it is
 * diagonal.  Each "point" of the plan is then one real coefficient of a field in a basis
 * of Laplace eigenfunctions (for example the real and imaginary parts of the discrete
 * Fourier coefficients), and kappa must be the same at every point (it may change in
 * time).  On such a coefficient -eps Laplace is the number eps |xi|^2, and the step is the
 * pointwise one with 1/De replaced by 1/De + rate[p]: the relaxation term of A and the
 * spatial term act alike.  The mass mode Phi_000 = 1 is the constant function, so its
 * source term zeta^{n+1} S(kappa~) reaches only the coefficient of the constant basis
 * function.
 *
 * rate          device [stride] FP64 (eps |xi|^2 of each point's basis function), or NULL
 *               for none.  Caller-owned; it must stay valid while steps are launched.
 * source_point  the point that holds the constant basis function's coefficient (it alone
 *               gets the mass-mode source), or -1: every point gets it (the plain
 *               pointwise form).
 * Applies to tfs_step, tfs_step_levels and tfs_step_adjoint (either scheme) until it is
 * called again; rate = NULL with source_point = -1 restores the pointwise form.
 * With a rate field the adjoint also accumulates sum_p rate_p dL/drate_p
 * (tfs_pbar_rate_gradient): for rate = eps |xi|^2 that is eps dL/deps.  The diagnostics'
 * minors do not describe a conformation tensor in this form; TFS_FLAG_CHECK_SYNC then
 * checks only the non-finite count.
 * Errors: TFS_EINVAL (null plan, source_point < -1 or >= npoints), TFS_EUNSUPPORTED (a rate
 * or a source point on a plan with FP32 velocity gradients).
 */
tfs_status tfs_plan_set_spatial(tfs_plan plan, const double* rate, int64_t source_point);

/*
 * Fourier layout of the spatial form on a periodic box (Sec. 4.1, eq. FP_discrete with
 * L = -eps Laplace - A(kappa~)): the basis tfs_plan_set_spatial takes, its rate field and
 * the changes of basis before and after a run.
 *
 * A box of shape[0..dim-1] grid points (C order, last axis fastest), N = n_0 ... n_{d-1}
 * of them, and extent[0..dim-1] lengths.  A real grid field f has the half spectrum
 *     F_q = (1/N) sum_x f(x) exp(-i xi_q . x),
 * q in C order over n_0 x ... x n_{d-2} x (n_{d-1}/2 + 1), so the zero wave vector holds
 * the mean.  Coefficient q takes the points 2q (real part) and 2q + 1 (imaginary part):
 * npoints = 2 n_0 ... n_{d-2} (n_{d-1}/2 + 1).  Integer wave numbers run 0, 1, .., -1 on the
 * leading axes (the Nyquist index of an even axis reads -n/2) and 0 .. n/2 on the last;
 * xi_j = 2 pi k_j / L_j.  Point 0, the constant function's coefficient, is the source
 * point.  The way back sums F_q exp(i xi_q . x) over the whole spectrum, the missing half
 * being the complex conjugate.  It assumes coefficients of a real field, conjugate-symmetric
 * where the half spectrum holds both partners (the planes of zero and Nyquist wave number
 * on the last axis); the steps of tfs_plan_set_spatial keep that symmetry, since both
 * partners of a pair see the same rate and the source reaches only the real part of the
 * zero wave vector.
 *
 * The object owns hipFFT (rocFFT) plans for one plane and a one-plane work buffer, both
 * made at creation; the conversions allocate nothing.  Each call runs asynchronously on the
 * stream it is given (a hipStream_t, NULL = default stream); calls on one object that
 * overlap in time (several streams or threads) race on the work buffer.
 */
typedef struct tfs_spectral_s* tfs_spectral;

/* Errors: TFS_EINVAL (dim not 2 or 3, null shape, extent or out, an axis outside 2 .. 2^20
 * points, an extent not finite and > 0, more than 2^30 points), TFS_ENOMEM, TFS_EHIP (hipFFT
 * plan creation included).  *out is NULL on error. */
tfs_status tfs_spectral_create(int dim, const int64_t* shape, const double* extent, tfs_spectral* out);

/* Release the object (NULL is accepted); synchronises the device first. */
tfs_status tfs_spectral_destroy(tfs_spectral s);

/* npoints of the layout (-1 for NULL). */
int64_t tfs_spectral_npoints(tfs_spectral s);

/*
 * The rate field of tfs_plan_set_spatial: rate[2q] = rate[2q + 1] = eps |xi_q|^2, and zero
 * at points npoints .. stride - 1.
 * rate  device [stride] FP64, caller-owned.
 * Errors: TFS_EINVAL (null object or rate, eps not finite and >= 0, stride < npoints).
 */
tfs_status tfs_spectral_rate(tfs_spectral s, double eps, double* rate, int64_t stride, void* stream);

/*
 * Grid fields to coefficients.
 * grid    device [nfields][grid_stride] FP64 (grid_stride >= N), read only.
 * points  device [nfields][point_stride] FP64 (point_stride >= npoints); points npoints ..
 *         point_stride - 1 of each plane are left as they are.  It must not overlap grid.
 * nfields 0 does nothing.
 * Errors: TFS_EINVAL (null object, nfields < 0, a null buffer with nfields > 0, a stride too
 * small), TFS_EHIP.
 */
tfs_status tfs_spectral_to_points(tfs_spectral s, const double* grid, int64_t nfields, int64_t grid_stride,
                                  double* points, int64_t point_stride, void* stream);

/*
 * Coefficients to grid fields, the inverse of tfs_spectral_to_points.
 * points  device [nfields][point_stride] FP64 (point_stride >= npoints), read only.
 * grid    device [nfields][grid_stride] FP64 (grid_stride >= N); grid points N ..
 *         grid_stride - 1 of each plane are left as they are.  It must not overlap points.
 * Errors as tfs_spectral_to_points.
 */
tfs_status tfs_spectral_to_grid(tfs_spectral s, const double* points, int64_t nfields, int64_t point_stride,
                                double* grid, int64_t grid_stride, void* stream);

/*
 * Analytic velocity gradient for fused launches: a sum of Fourier terms on the periodic
 * grid [0, 2 pi)^d with `grid` points per axis,
 *     kappa_ij(x, t) = sum_n coef[n][i][j] sin(k[n] . x + phase[n] + omega[n] t),
 * x_a = 2 pi idx_a / grid, the plan's point p being the flat grid index point0 + p with
 * idx_0 varying fastest.  A divergence-free field u = sum_n A_n e_n cos(k_n . x + ...) has
 * coef[n][i][j] = -A_n e_n,i k_n,j.  All arrays are host memory, copied (the plan owns the
 * device copy; the call allocates and synchronises the plan's stream).
 */
#define TFS_FIELD_MAX_TERMS 4096
typedef struct tfs_field {
    int32_t nterms;            /* number of terms, 0 .. TFS_FIELD_MAX_TERMS (0: kappa = 0) */
    int64_t grid;              /* grid points per axis */
    int64_t point0;            /* flat grid index of the plan's point 0 */
    const double* k;           /* [nterms][d] wave vectors */
    const double* phase;       /* [nterms] */
    const double* omega;       /* [nterms] angular frequencies (all zero: a steady field) */
    const double* coef;        /* [nterms][d][d] */
} tfs_field;

/* Errors: TFS_EINVAL (null plan or field, nterms out of range, grid < 1, the points outside
 * the grid, a null or non-finite table), TFS_ENOMEM, TFS_EHIP. */
tfs_status tfs_plan_set_field(tfs_plan plan, const tfs_field* field);

/*
 * The plan's analytic velocity gradient (tfs_plan_set_field) at time t on the plan's points,
 * written for the step calls: kappa_out[q][p] = kappa_q(x_p, t) + add[q][p], the sums in FP64,
 * rounded once to the plan's kappa precision.  With integer wave vectors (and grid + nterms
 * <= 2048) each term's sine is a root of unity of the grid, e^{2 pi i (k . idx mod grid)/grid},
 * times the term's e^{i (phase + omega t)}: the phase is reduced exactly, within a few ulp of
 * the field; otherwise the sine of each term's FP64 phase (whose rounding, |k . x| 2^-53, is
 * the error there).  This is
 * input synthesis for callers whose gradient is that field (the benchmark workloads); the
 * update itself never calls it.
 * add        device [d*d][stride] FP64 (a steady perturbation of the field), or NULL.
 * kappa_out  device [d*d][stride] in the plan's kappa precision; columns >= npoints untouched.
 * Asynchronous on the plan's stream; no allocation.
 * Errors: TFS_EINVAL (null plan, no field set, non-finite t, null kappa_out), TFS_EHIP.
 */
tfs_status tfs_field_eval(tfs_plan plan, double t, const double* add, void* kappa_out);

/*
 * Temporally fused steps: advance every point from level n0 to n0 + nsteps in ONE launch,
 * with kappa evaluated from the plan's field inside the kernel at t_n = n dt, as tfs_step
 * would advance them with those kappa levels:
 *   TFS_SCHEME_EXP   kappa~ = 3/2 kappa(t_n) - 1/2 kappa(t_{n-1}) (kappa(t_0) at n = 0);
 *   TFS_SCHEME_BDF2  kappa~ = 2 kappa(t_n) - kappa(t_{n-1}) (eq. BDF_and_extrapolation), from
 *                    n0 >= 1: level 0 -> 1 is the SDIRK2 start, taken with tfs_step.
 * Each point's mode levels, X and kappa stay in registers for all nsteps steps: HBM is read
 * once and written once per launch.
 *
 * X    device [2][c][stride] ring: levels n0 (slot n0 % 2) and, for BDF2, n0 - 1 on entry; on
 *      return level n0 + nsteps in slot (n0 + nsteps) % 2 and level n0 + nsteps - 1 in the
 *      other slot.
 * Y    device modes in the plan's layout (Y_k = X_k - c_k X): for BDF2 the two-slot ring of
 *      tfs_step, for EXP its one level, updated in place (ignored on entry when n0 = 0).
 * tau  device [c][stride] or NULL: tau at level n0 + nsteps.
 * Asynchronous on the plan's stream; no allocation.  Requires m = 16 or 32 (FP32 modes in
 * 3-D; either precision in 2-D), no spatial form, and a field.
 * Errors: TFS_EINVAL (null plan, no field, 0 <= n0 <= n0 + nsteps <= max_steps violated, a
 * BDF2 launch from n0 = 0, null X or Y), TFS_EUNSUPPORTED (other m or precision, or a
 * spatial form), TFS_EHIP.
 */
tfs_status tfs_run_fused(tfs_plan plan, int64_t n0, int64_t nsteps, double* X, void* Y, double* tau);

/*
 * Advance every point from time level n to n+1 (0 <= n < max_steps), asynchronously
 * on the plan's stream; no allocation, no host synchronisation (unless
 * TFS_FLAG_CHECK_SYNC).
 *
 * kappa_a, kappa_b  device [d*d][stride] in the plan's kappa precision (FP64, or FP32 with
 *                   TFS_KAPPA_FP32).  The step is driven by
 *                   kappa~ = 2 kappa_a - kappa_b  (second-order extrapolation
 *                   E^{n+1} kappa = 2 kappa^n - kappa^{n-1}, eq. BDF_and_extrapolation:
 *                   pass kappa^n, kappa^{n-1}), or kappa~ = kappa_a when kappa_b is NULL
 *                   (pass the gradient of the already updated velocity kappa^{n+1}, as in
 *                   eq. FP_discrete).  At n = 0 kappa_b is ignored.
 * X                 device [L][c][stride] FP64 ring, L = tfs_plan_x_levels (2, or 3 for the
 *                   shifted mode form): slot j%L holds level j.  The caller stores X^0 in
 *                   slot 0 before n = 0.  Level n+1 overwrites slot (n+1)%L.
 * Y                 device ring of the fractional modes, 2 * m * c * stride elements in the
 *                   plan's (possibly tiled) layout, in the plan's mode form (tfs_mode_form;
 *                   FP64, or FP32 for TFS_FP32_MODES): slot j%2 holds level j.  Written
 *                   entirely at n = 0 (levels 0 and 1); its input contents are ignored then.
 * tau               device [c][stride] FP64 or NULL: tau^{n+1} = gamma D^{1-alpha} X^{n+1}.
 * diag              device [6] FP64 or NULL: over the points at level n+1, the minimum of the
 *                   three leading principal minors of C = I + X (Sylvester's criterion as used
 *                   in the appendix; in 2-D the third equals the second), max ||tau||_F,
 *                   sum ||tau||_F^2 (full tensor), and the count of non-finite X or tau
 *                   entries.  Minima and maxima skip non-finite values.
 * Errors: TFS_EINVAL (null plan/X/Y/kappa_a, n out of range, diag requested with
 * npoints == 0 is fine), TFS_EHIP, TFS_ENUMERIC (only with TFS_FLAG_CHECK_SYNC).
 *
 * TFS_SCHEME_EXP plans: kappa~ = (3/2) kappa_a - (1/2) kappa_b (kappa^n, kappa^{n-1}
 * extrapolated to the half step), or kappa_a when kappa_b is NULL or n = 0.  X is the same
 * ring (only level n is read).  Y holds ONE level, m * c * stride elements in the plan's
 * layout, in the representation Y_k = X_k - q_k X with q_k = w_k dt a1_k, updated in place
 * from level n to n+1; at n = 0 its input contents are ignored (the modes start at zero).
 */
tfs_status tfs_step(tfs_plan plan, int64_t n, const void* kappa_a, const void* kappa_b,
                    double* X, void* Y, double* tau, double* diag);

/*
 * tfs_step for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same arguments, kernels and results, but
 * the diagnostics' block partials (the step's only scratch) live in a static device array of the
 * library, 8192 partials (384 KiB) per device, held until the process ends, instead of the
 * plan's buffer.  The call allocates and frees nothing.  The array's address on the device is
 * looked up once per device at tfs_plan_create.
 * Limit: with diag, the step's launches write up to 2 x CUs x grid_per_cu partials; a plan above
 * 8192 (more than 16 blocks per CU on a 256-CU device, see tfs_plan_tune) is refused with
 * TFS_EINVAL before anything is launched.  Without diag it is tfs_step.
 * Every call on a device shares that device's array (each launch writes the partials it reads
 * before reading them, so nothing carries over between calls); calls that overlap in time on
 * one device, on different streams or from different threads, race on it.
 * Errors: those of tfs_step, and TFS_EHIP if the array's address could not be looked up.
 */
tfs_status tfs_step_noalloc(tfs_plan plan, int64_t n, const void* kappa_a, const void* kappa_b,
                            double* X, void* Y, double* tau, double* diag);

/*
 * tfs_step with explicit time levels instead of the two-slot rings, so that a caller can
 * keep every level (checkpointed recomputation for the adjoint).  Same update, same
 * layouts per level:
 *   X_n, X_nm1, X_out    [c][stride] FP64: levels n, n-1 (unused at n = 0) and n+1;
 *                        X_out must not alias X_n (it may alias X_nm1).
 *   X_nm2                [c][stride] FP64 level n-2: read by shifted-mode-form plans at n >= 2
 *                        (X_out may alias it); ignored otherwise.
 *   Y_n, Y_nm1, Y_out    m * c * stride mode elements each (plan precision and tiling):
 *                        levels n, n-1 and n+1; Y_out may alias Y_nm1 but not Y_n.
 *                        At n = 0 the start-up writes level 0 into Y_nm1 and level 1 into
 *                        Y_out, and Y_n is unused.
 * Errors as tfs_step, plus TFS_EINVAL for the forbidden aliases.
 * TFS_SCHEME_EXP plans read X_n and Y_n (ignored at n = 0) and write X_out and Y_out,
 * which may alias Y_n; X_nm1 and Y_nm1 are unused.
 */
tfs_status tfs_step_levels(tfs_plan plan, int64_t n, const void* kappa_a, const void* kappa_b,
                           const double* X_n, const double* X_nm1, const double* X_nm2, double* X_out,
                           const void* Y_n, void* Y_nm1, void* Y_out, double* tau, double* diag);

/*
 * Adjoint of one step (reverse mode), for a scalar loss L of the stresses.  The forward
 * BDF2 step and the SDIRK2 start-up are linear in (X, Y); this call applies the transpose of
 * step n -> n+1 and accumulates the gradients of the step's coefficients.  It is the
 * derivative of the scheme of Sec. 4.1; the paper itself does not differentiate it.
 *
 * Call it for n = N-1, N-2, ..., 0 after zeroing Xbar and Hbar, with the forward levels of
 * the same run (recomputed from checkpoints by the caller):
 *   X_n, X_nm1, X_np1   [c][stride] FP64 forward levels n, n-1, n+1 (X_n = X^0 at n = 0;
 *                       X_nm1, X_np1 unused at n = 0)
 *   X_nm2               forward level n-2: read by shifted-mode-form plans at n >= 2 only
 *   Y_n, Y_nm1          forward mode levels n, n-1 (tiled layout; unused at n = 0)
 *   kappa_a, kappa_b    as passed to the forward step n (the plan's kappa precision)
 *   Xbar                device [L][c][stride] FP64 adjoint ring (L = tfs_plan_x_levels).  With
 *                       L = 2: before step n, slot (n+1)%2 holds dL/dX^{n+1} from the later
 *                       steps and slot n%2 the part of dL/dX^n from step n+1; after it, slot n%2
 *                       holds dL/dX^n complete and slot (n+1)%2 the part of dL/dX^{n-1} from
 *                       step n.  With L = 3 (the shifted mode form, where step n also reads
 *                       X^{n-2}): before step n, slot (n+1)%3 holds dL/dX^{n+1} complete, slot
 *                       n%3 and slot (n-1)%3 the parts of dL/dX^n and dL/dX^{n-1} from the later
 *                       steps (zero before the last step); after it, slot n%3 holds dL/dX^n
 *                       complete, slot (n-1)%3 the part of dL/dX^{n-1} so far and slot (n+1)%3
 *                       the part of dL/dX^{n-2} from step n.  After n = 0, slot 0 is dL/dX^0.
 *   Hbar                device mode-adjoint ring (2 slots, plan precision and tiling) holding
 *                       H_k^(j) = dL/d(2 Y_k^j - Y_k^{j-1}/2); slot j%2 holds H^(j).
 *   taubar              device [c][stride] FP64 dL/dtau^{n+1} (or NULL: no direct loss on it)
 *   kappabar_a/_b       device [d*d][stride] FP64, accumulated: dL/dkappa_a, dL/dkappa_b of
 *                       this step (NULL to skip).  Passing the same buffer for both gives the
 *                       derivative with respect to a kappa shared by both arguments.
 *   pbar                device [tfs_pbar_size] FP64, accumulated: gradients of the per-mode
 *                       factors, the scalar factors and zeta^{n+1}; convert with
 *                       tfs_pbar_to_params.
 * TFS_SCHEME_EXP plans: X_nm1 and Y_nm1 are unused (X_np1 is read at every n, Y_n for
 * n >= 1); Xbar is the same ring (slot (n+1)%2 holds dL/dX^{n+1} complete, slot n%2
 * receives dL/dX^n), and Hbar is a single mode level holding dL/dY^{n+1} before the call and
 * dL/dY^n after it.
 * Asynchronous on the plan's stream.  Errors: TFS_EINVAL (null required pointer, n out of
 * range), TFS_EHIP.
 */
tfs_status tfs_step_adjoint(tfs_plan plan, int64_t n, const void* kappa_a, const void* kappa_b,
                            const double* X_n, const double* X_nm1, const double* X_nm2, const double* X_np1,
                            const void* Y_n, const void* Y_nm1, double* Xbar, void* Hbar,
                            const double* taubar, double* kappabar_a, double* kappabar_b, double* pbar);

/* Length of the pbar accumulator of a plan: 6 m + 16 + max_steps + 1. */
int64_t tfs_pbar_size(tfs_plan plan);

/*
 * Host chain rule from an accumulated pbar (host copy) to the gradients with respect to the
 * weights and poles (dL_dw, dL_dlambda: host [m]), the relaxation time De and eta_p (host
 * scalars), through every coefficient the plan derived from them: the BDF2 factors, the
 * SDIRK2 start-up factors and the mass-mode memory table (of the exponential-mode factors and
 * its mass-mode increments for TFS_SCHEME_EXP plans), and on to the fractional order:
 *   dL_dalpha = sum_k (dL/dw_k dw_k/dalpha + dL/dlambda_k dlambda_k/dalpha)   (compensated),
 * with dw_dalpha, dlambda_dalpha (host [m]) the derivatives of the plan's sum-of-exponentials
 * rule, for example those tfs_soe_gl_log returns for a window held fixed (Sec. 2.2).
 * Any output may be NULL; dw_dalpha and dlambda_dalpha are read only for dL_dalpha.
 * Errors: TFS_EINVAL (null plan or pbar, dL_dalpha without both derivative tables).
 */
tfs_status tfs_pbar_to_params(tfs_plan plan, const double* pbar_host, const double* dw_dalpha,
                              const double* dlambda_dalpha, double* dL_dw, double* dL_dlambda,
                              double* dL_dDe, double* dL_deta_p, double* dL_dalpha);

/*
 * Spatial form: sum_p rate_p dL/drate_p from a host copy of the accumulated pbar of a
 * backward pass (eps dL/deps when rate = eps |xi|^2: the gradient with respect to the
 * diffusion coefficient, scaled).  Zero without a rate field.
 * Errors: TFS_EINVAL (null plan, pbar or out).
 */
tfs_status tfs_pbar_rate_gradient(tfs_plan plan, const double* pbar_host, double* out);

/*
 * Plain fractional modes X_k of time level `level` from the rings of tfs_step: the mode
 * ring's slot level%2 and the X ring's levels `level` and `level`-1 (X_k = Y_k + c_k X^level,
 * plus beta_k X^{level-1} in the shifted form, X^{-1} = 0), the latter two still in the X ring.
 * Xk_out: device [m][c][stride] FP64, untiled.  Asynchronous on the plan's stream.
 * TFS_SCHEME_EXP plans: Y is the single mode level, holding level `level`; X_k = Y_k + q_k X.
 * Errors: TFS_EINVAL (null plan, level < 0).
 */
tfs_status tfs_modes_to_plain(tfs_plan plan, int64_t level, const double* X, const void* Y, double* Xk_out);

/* Slots of the plan's X ring (and of the adjoint's Xbar ring): 2, or 3 for the shifted mode form. */
int32_t tfs_plan_x_levels(tfs_plan plan);

/*
 * Host copies of the plan's coefficient tables, FP64:
 *   tables  [5][m]: d_k, c_k, eta_k, u_k, v_k (u_k, v_k: SDIRK2 start-up mode factors)
 *   scalars [8]:    eta, sum_k eta_k c_k, b0 + eta/De, gamma/dt, theta, rho, sigma1, sigma2
 *   zeta    [max_steps+1]: zeta^j (zeta^0 = zeta^1 = 0 are unused)
 * Any pointer may be NULL.  TFS_SCHEME_EXP plans: tables e_k, q_k, lambda_k dt, 1 - e_k,
 * w_k dt a0_k; scalars q = sum_k q_k, sum_k ((1 - e_k) q_k - w_k dt a0_k), 1 + q/De,
 * gamma/dt, dt sum_k (w_k - lambda_k q_k), 0, 0, 0; zeta^{n+1} = sum_k (mu_k^{n+1} - mu_k^n).
 */
tfs_status tfs_plan_tables(tfs_plan plan, double* tables, double* scalars, double* zeta);

/* Effective plane stride (elements) of the plan. */
int64_t tfs_plan_stride(tfs_plan plan);

/* Mode-ring tile of the plan (points; 0 = untiled). */
int64_t tfs_plan_tile(tfs_plan plan);

/*
 * Launch tuning; does not change results beyond rounding-order-free choices:
 *   "vec"          points per lane: 0 = widest width the alignment of the fields allows up
 *                  to 2 (4 for 2-D TFS_FP32_MODES plans) (default), or 1, 2 (and 4 for
 *                  TFS_FP32_MODES); a width the alignment does not allow falls back to 1 at launch.
 *   "adj_vec"      points per lane of the BDF2 adjoint: 0 (default: 2 for FP32 modes, 1 for FP64), 1 or 2.
 *   "grid_per_cu"  cap on blocks per compute unit of the grid-stride launches, 1..64 (default:
 *                  1 for TFS_FP64 plans, 16 for TFS_FP32_MODES plans).
 * Note: the diagnostic sum's rounding order depends on the grid; results of X, tau, Y do not.
 */
tfs_status tfs_plan_tune(tfs_plan plan, const char* key, int64_t value);

/*
 * Sum-of-exponentials fit of t^(alpha-1)/Gamma(alpha) with exactly m modes, host, FP64.
 * The Laplace symbol s^(-alpha) = (sin(pi alpha)/pi) int exp((1-alpha)y)/(s+e^y) dy is
 * discretised in y = ln(lambda): one lambda = 0 mode for y < y_lo, an (m-2)-point
 * Gauss-Legendre rule on [y_lo, y_hi], one mode lambda = e^{y_hi}(1+alpha)/alpha carrying
 * the mass and first moment of y > y_hi.  w_k > 0, lambda_k >= 0 by construction, so the
 * approximate kernel is completely monotone (Sec. 2.2).  The window minimises the
 * relative error of the symbol on [0.1/T, 10/dt].  alpha = 1 gives w = (1, 0, ...), lambda = 0.
 * Outputs (host, [m] each; dw_dalpha/dlambda_dalpha may be NULL): derivatives at the
 * fixed window.  info (host [4] or NULL): y_lo, y_hi, symbol relative error, time-domain
 * relative error on [dt, T].
 * Errors: TFS_EINVAL (alpha not in (0,1], m < 1, dt <= 0, T <= dt, null w/lambda).
 */
tfs_status tfs_soe_fit(double alpha, int32_t m, double dt, double T, double* w, double* lambda,
                       double* dw_dalpha, double* dlambda_dalpha, double* info);

/* Same rule at a given window (y_lo < y_hi). */
tfs_status tfs_soe_gl_log(double alpha, int32_t m, double y_lo, double y_hi, double* w, double* lambda,
                          double* dw_dalpha, double* dlambda_dalpha);

/* Static description of a status code. */
const char* tfs_status_string(tfs_status s);

/* Thread-local text of the last error reported by this library ("" if none). */
const char* tfs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TFS_H */

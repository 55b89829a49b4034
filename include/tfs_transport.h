/*
 * tfs_transport.h -- C ABI of the stress update with the transport terms of the MFP
 * equation on a periodic grid (Sec. 4.1, eq. FP_discrete with L = u.grad - eps Laplace -
 * A(kappa~)): advection by a velocity field u(x) and centre-of-mass diffusion, both inside
 * the implicit operator (b_0 + eta L) of the BDF2 scheme and of its SDIRK2 start, with u and
 * kappa varying in space and time.
 *
 * The operator couples the points, so a step is no longer pointwise.  Per step:
 *   1. the modes advance pointwise (in the Y-form of tfs.h they do not depend on X^{n+1});
 *      each point's right-hand side R and history combination G come out of the same pass;
 *   2. the right-hand side gains L's transport part applied to G (the history terms
 *      sum_k eta_k L Phi_k of eq. FP_discrete);
 *   3. the coupled system (a I - b K(kappa~(x)) + b T) X = rhs, T = u~.grad - eps Laplace, is
 *      solved by a fixed number of splitting iterations (or GMRES steps,
 *      tfs_transport_set_method) preconditioned by its constant-coefficient part: with the
 *      spatial means kappa_bar and u_bar,
 *          P(xi) = (a + b eps |xi|^2 + i b xi.u_bar) I - b K(kappa_bar),
 *          X_hat <- P^{-1} (rhs_hat - F[ -b K(kappa~ - kappa_bar) X + b (u~ - u_bar).grad X ]),
 *      which converges when the variable part is small next to P (small dt, eps > 0 or a
 *      nearly uniform u);
 *   4. tau from X^{n+1} and G, pointwise.
 * The SDIRK2 start solves the same kind of system once per stage.  With a TFS_SCHEME_EXP plan
 * (the exponential-mode extension) the state takes the increment form
 * X^{n+1} - X^n = -L sum_k (X_k^{n+1} - X_k^n) of that scheme: step 1 gives R and H
 * (sum_k (X_k^{n+1} - X_k^n) = q X^{n+1} - H), the right-hand side gains T H, and step 3 solves
 * ((1 + q/De) I - q K(kappa~) + q T) X = rhs; there is no start-up step.  Derivatives are spectral
 * (first derivatives with the Nyquist wave number taken as zero); transforms are hipFFT
 * plans made at creation.
 *
 * Layouts: as tfs.h (grid fields [comp][stride], point index = C-order grid index); the
 * velocity u is [d][stride] FP64.  The object owns its FFT plans and work buffers (about
 * (6c + 2cd) planes of the stride plus spectral planes), allocated at creation.
 */
#ifndef TFS_TRANSPORT_H
#define TFS_TRANSPORT_H

#include <stdint.h>

#include "tfs.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tfs_transport_s* tfs_transport;

/*
 * A periodic box of shape[0..dim-1] points (each >= 2) and extent[0..dim-1] lengths (> 0),
 * centre-of-mass diffusion eps >= 0, grid fields of plane stride `stride` (the stress plan's
 * stride), and `iters` >= 0 splitting iterations per solve (0: the preconditioner alone,
 * exact when kappa and u are uniform).
 * Errors: TFS_EINVAL, TFS_ENOMEM, TFS_EHIP.  *out is NULL on error.
 */
tfs_status tfs_transport_create(int dim, const int64_t* shape, const double* extent, double eps, int64_t stride,
                                int iters, tfs_transport* out);

/* Release (NULL is accepted); synchronises the device first. */
tfs_status tfs_transport_destroy(tfs_transport tr);

/*
 * Transform form, as tfs_ns_batched / tfs_ns_set_batched: 1 when whole fields go through
 * batched hipFFT plans (tried at creation), 0 when planes go one at a time; set_batched(0)
 * forces planes one at a time, set_batched(1) asks for the batched plans (TFS_EUNSUPPORTED
 * if hipFFT refuses the layout).  Results agree to rounding.
 */
int tfs_transport_batched(tfs_transport tr);
tfs_status tfs_transport_set_batched(tfs_transport tr, int on);

/*
 * The solver of step 3: method 0 (the default) runs `iters` splitting iterations; method 1
 * runs GMRES on the same preconditioned system (the splitting's fixed-point equation
 * (I + N) x = b, real inner product over the coefficients) with at most `iters` Arnoldi steps
 * from zero, stopping early at a relative residual of 1e-15.  The basis is built with N, whose
 * Krylov space is that of I + N, and one is added to the Hessenberg matrix's diagonal
 * (classical Gram-Schmidt, with a second pass where the first cancels more than half of the
 * vector's squared norm).  GMRES converges
 * where the splitting contracts slowly or not at all (strong advection, small eps).  Its
 * least-squares problem (Hessenberg matrix, Givens rotations, residual test, back
 * substitution) stays on the device, so the Arnoldi steps are queued without waiting; the
 * host reads the residual test every `every` steps (tfs_transport_set_tolerance) to stop
 * early.  It keeps iters + 1 basis vectors of 2 c nc doubles (allocated here).
 * Errors: TFS_EINVAL (null object, unknown method, iters > 256 for GMRES), TFS_ENOMEM.
 */
tfs_status tfs_transport_set_method(tfs_transport tr, int method);

/*
 * Early exit of the solves: with tol > 0 the splitting stops once an iteration changes the
 * coefficients by at most tol relative to their norm, and GMRES once its relative residual is
 * at most tol; both are tested on the host every `every` iterations (one stream
 * synchronisation per test; the default is 5); `iters` stays the cap.  tol = 0 (the default)
 * restores the fixed counts (GMRES still stops at 1e-15, seen every `every` steps).
 * Errors: TFS_EINVAL (null object, tol < 0 or not finite, every < 1).
 */
tfs_status tfs_transport_set_tolerance(tfs_transport tr, double tol, int every);

/* Iterations (or Arnoldi steps) the longest solve of the last tfs_transport_step took; -1
 * for a null object. */
int tfs_transport_last_iterations(tfs_transport tr);

/*
 * One step n -> n+1 with the transport terms: as tfs_step (the same X and Y rings and
 * levels; for TFS_SCHEME_BDF2 plans SDIRK2 at n = 0 and BDF2 after, for TFS_SCHEME_EXP plans
 * the exponential-mode step at every n), with the velocity levels u_a, u_b [d][stride]
 * following kappa's rule (extrapolated 2 u_a - u_b, or 3/2 u_a - 1/2 u_b for the exponential
 * scheme, when kappa_b is given and n >= 1, else u_a).  The plan must match the object (dim,
 * npoints, stride) and be pointwise (no tfs_plan_set_spatial).  diag (device [6] FP64, or
 * NULL) receives tfs_step's diagnostics of level n+1; TFS_FLAG_CHECK_SYNC acts as in
 * tfs_step.
 * Errors: TFS_EINVAL (null or mismatched arguments, u_b missing while kappa_b is given),
 * TFS_EUNSUPPORTED (spatial form), TFS_EHIP, TFS_ENUMERIC (only with TFS_FLAG_CHECK_SYNC).
 */
tfs_status tfs_transport_step(tfs_transport tr, tfs_plan plan, int64_t n, const double* kappa_a,
                              const double* kappa_b, const double* u_a, const double* u_b, double* X, void* Y,
                              double* tau, double* diag);

#ifdef __cplusplus
}
#endif

#endif

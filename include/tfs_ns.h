/*
 * tfs_ns.h -- C ABI of the coupled step: the incompressible Navier-Stokes equations on a
 * periodic box (Sec. 2, eq. Navier_Stokes)
 *
 *   du/dt + (u . grad) u + grad p - nu Laplace u = div tau,   div u = 0,   nu = beta/Re,
 *
 * advanced by the projection method of Sec. 4.1 (eqs. BDF_and_extrapolation,
 * velocity_correction, time_discretization_NS, NS_Poisson, NS_Helmholtz) and coupled to the
 * stress update of tfs.h: a step first computes the velocity of level n+1 from levels n and
 * n-1 and the extrapolated explicit term E^{n+1}(-(u.grad)u + div tau), then calls
 * tfs_step with kappa^{n+1} = grad u^{n+1} (no extrapolation of kappa: the gradient of the
 * already updated velocity), which advances X, the modes and tau to level n+1.
 *
 * Space is pseudo-spectral.  On a periodic box the pressure Poisson and velocity Helmholtz
 * equations are Fourier multipliers: with R = -sum_j (b_j/dt) u^{n+1-j} + E^{n+1}(F),
 * F = -(u.grad)u + div tau, the pressure is p = -i xi . R / |xi|^2 (mean zero) and
 *     u^{n+1} = (R - xi (xi . R)/|xi|^2) / (b_0/dt + nu |xi|^2),
 * the curl-curl part of the explicit term having no divergence.  Products are formed on
 * the grid, derivatives as i xi; the explicit term and the initial velocity keep only the
 * 2/3 band |k_j| < n_j/3 of integer wave numbers, so the quadratic term is alias-free and
 * the Nyquist modes stay empty.  Transforms are hipFFT (rocFFT) plans made at creation.
 * g = 1 (BDF1, E f = f^n) at the first step, g = 2 (b = (3/2, -2, 1/2), E f = 2 f^n - f^{n-1})
 * after.  The stress update is tfs.h's pointwise model, or with tfs_ns_set_transport the MFP
 * equation with its advection and diffusion terms (tfs_transport.h).
 *
 * Layouts (all device memory, caller-owned, FP64):
 *   grid fields    structure-of-arrays, point index = C-order index of the grid point
 *                  (last axis fastest), plane stride `stride` (the stress plan's stride):
 *                  u [d][stride], kappa [d*d][stride] (kappa_ij = d u_i/d x_j at i*d+j),
 *                  and the plan's X, Y, tau.
 *   coefficients   the half spectrum of a real field: nc = n_0 ... n_{d-2} (n_{d-1}/2 + 1)
 *                  complex numbers (re, im interleaved), C order, normalised so that the
 *                  zero wave vector holds the mean.  uh [2][d][nc] is the velocity ring
 *                  (level n in slot n % 2), fh [2][d][nc] the ring of explicit terms
 *                  (F^n in slot n % 2).
 * The object owns its FFT plans and work buffers (allocated at creation, never by a step).
 * A step runs on the stress plan's stream.
 */
#ifndef TFS_NS_H
#define TFS_NS_H

#include <stdint.h>

#include "tfs.h"
#include "tfs_transport.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tfs_ns_s* tfs_ns;

/*
 * Create the velocity solver of a periodic box of shape[0..dim-1] points (each >= 2) and
 * extent[0..dim-1] lengths (> 0), viscosity nu = beta/Re >= 0, step dt > 0, for grid fields
 * of plane stride `stride` (>= the number of points; pass the stress plan's stride).
 * Errors: TFS_EINVAL (dim not 2/3, bad sizes), TFS_ENOMEM, TFS_EHIP (hipFFT plan
 * creation included).  *out is NULL on error.
 */
tfs_status tfs_ns_create(int dim, const int64_t* shape, const double* extent, double nu, double dt,
                         int64_t stride, tfs_ns* out);

/* Release the solver (NULL is accepted); synchronises the device first. */
tfs_status tfs_ns_destroy(tfs_ns ns);

/* nc: complex coefficients per velocity component (the half-spectrum size). */
int64_t tfs_ns_spectral_size(tfs_ns ns);

/*
 * 1 when the solver transforms whole fields in batched hipFFT plans, 0 when it transforms
 * one plane at a time (hipFFT refuses the batched layout, planes `stride` apart, for some
 * sizes; the results are the same).
 */
int tfs_ns_batched(tfs_ns ns);

/*
 * Choose the transform form: on = 0 transforms one plane at a time, on = 1 asks for the
 * batched plans (the form tfs_ns_create tries first).  Synchronises the device and remakes
 * the plans.  Errors: TFS_EINVAL (null solver), TFS_EUNSUPPORTED (on = 1 and hipFFT
 * refuses the batched layout; the solver then transforms one plane at a time), TFS_EHIP.
 */
tfs_status tfs_ns_set_batched(tfs_ns ns, int on);

/*
 * Stress update of the coupled step: tr = NULL (the default) uses tfs_step, the pointwise
 * update; otherwise tfs_transport_step(tr, plan, n, kappa^{n+1}, NULL, u^{n+1}, NULL, ...),
 * which adds the MFP equation's advection by u and centre-of-mass diffusion (eq. FP_discrete
 * in full).  The solver keeps the handle; tr must outlive its use.  Errors: TFS_EINVAL (null
 * solver).
 */
tfs_status tfs_ns_set_transport(tfs_ns ns, tfs_transport tr);

/*
 * Level 0: from the grid velocity u [d][stride] (overwritten), keep its divergence-free
 * part in the 2/3 band (Sec. 4.1 asks for a solenoidal velocity), store its coefficients
 * in slot 0 of uh, and write u^0 and kappa^0 = grad u^0 back on the grid.  Runs on the
 * plan's stream; the plan (dim, npoints, stride) must match the solver and must not have
 * a spatial form set (tfs_plan_set_spatial: its points are Fourier coefficients).
 * Errors: TFS_EINVAL (null pointers, mismatched or spatial-form plan), TFS_EHIP.
 */
tfs_status tfs_ns_init(tfs_ns ns, tfs_plan plan, double* u, void* uh, double* kappa);

/*
 * One coupled step n -> n+1 (0 <= n < the plan's max_steps).  On entry u, kappa and tau
 * hold level n (tau = 0 at n = 0: the stress of level 0), uh holds levels n and n-1 (n-1
 * unused at n = 0) and fh slot (n-1) % 2 holds F^{n-1} (unused at n = 0).  The step writes
 * F^n to fh slot n % 2, u^{n+1} to uh slot (n+1) % 2, u and kappa of level n+1 on the grid,
 * and then calls tfs_step(plan, n, kappa, NULL, X, Y, tau, diag), or the transport step set
 * by tfs_ns_set_transport.
 * Errors: those of tfs_step, TFS_EINVAL (null pointers, mismatched or spatial-form plan),
 * TFS_EHIP.
 */
tfs_status tfs_ns_step(tfs_ns ns, tfs_plan plan, int64_t n, double* u, void* uh, void* fh, double* kappa,
                       double* X, void* Y, double* tau, double* diag);

#ifdef __cplusplus
}
#endif

#endif

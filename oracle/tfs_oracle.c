/*
 * CPU ORACLE — test infrastructure only.
 *
 * Plain, slow FP64 reference of the kernel-compressed time-fractional
 * macroscopic Fokker-Planck update, applied independently at every point of a
 * homogeneous-flow problem (the velocity gradient kappa is prescribed, there is
 * no spatial operator).  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library; the product path never does.
 *
 * It works in the paper's own variables: the Hermite spectral modes of degree 0
 * and 2 (Sec. 3.4, ordering of the vector Phi; 2-D ordering (00, 11, 02, 20)),
 * with the mass mode Phi_0 carried per point together with its own fractional
 * modes, plain fractional modes Phi_k (Sec. 4, eqs. for the approximate
 * macroscopic system), a full (c+1)x(c+1) system solved by Gaussian
 * elimination with partial pivoting, and Neumaier sums for the recombination.
 *
 * Readings taken where the paper is ambiguous (each is listed in the design
 * notes of the repository):
 *  - the coupling matrix is assembled from the tested configuration operator
 *    (Sec. 3.2, eq. conf_op_tested) with a = 1/sqrt(2), not from the printed
 *    block matrix of Sec. 3.4, which disagrees with it;
 *  - Hermite variables are normalised by the mass mode (Phi_0 = 1), so the
 *    Kramers stress (Sec. 2 and eq. ExtraStressN_0and2order, chi_0 = 0) is
 *    tau_ll = gamma*sqrt(2)*D_{2e_l}, tau_lm = gamma*D_{e_l+e_m} with
 *    D the kernel-compressed fractional derivative, gamma = eta_p/De;
 *  - the first step is Alexander's two-stage L-stable SDIRK2 on the
 *    augmented linear system (Sec. 5.1 asks for an SDIRK2 start), later steps
 *    are the BDF2 scheme of eqs. BDF_Phi_k_n+1 and FP_discrete;
 *  - BDF2 coefficients b = (3/2, -2, 1/2); second-order extrapolation
 *    E^{n+1} f = 2 f^n - f^{n-1} (eq. BDF_and_extrapolation).
 *
 * A second scheme (not the paper's; an extension of it) advances each mode by
 * the exact solution of the mode equation f_k' = -lam_k f_k + w_k f (Sec. 2.2)
 * over a step on which f is linear in time.  Since the kernel-compressed
 * derivative sum_k (w_k f - lam_k f_k) is sum_k f_k', the state equation
 * Phi' = A(kappa) sum_k Phi_k' is then integrated over the step as
 * Phi^{n+1} - Phi^n = A(kappa~) sum_k (Phi_k^{n+1} - Phi_k^n), exact for constant
 * kappa, with kappa~ at the half step (one-step scheme, no start-up step).
 *
 * The same source is compiled three times: with real doubles (orc_*), with C99
 * complex doubles (orcz_*) for complex-step derivatives (the imaginary part of
 * every output is the directional derivative along the imaginary part of the
 * inputs, exact to rounding), and with x87 extended-precision long doubles
 * (orcl_*, 64-bit significand) as a reference for the rounding error of FP64
 * evaluations of the same discrete scheme.  Branches compare real parts only.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#if defined(ORC_COMPLEX)
typedef double complex sc;
typedef double rl;       /* real scalar of the build */
#define ORC(name) orcz_##name
#define RE(x) creal(x)
#elif defined(ORC_LONG)
typedef long double sc;
typedef long double rl;
#define ORC(name) orcl_##name
#define RE(x) (x)
#else
typedef double sc;
typedef double rl;
#define ORC(name) orc_##name
#define RE(x) (x)
#endif

#ifdef ORC_LONG
#define SQRTR(x) sqrtl(x)
#define FABSR(x) fabsl(x)
#else
#define SQRTR(x) sqrt(x)
#define FABSR(x) fabs(x)
#endif

#define MAXD 3
#define MAXN 7 /* c + 1 in 3-D */

#if defined(ORC_COMPLEX)
#define EXPS(x) cexp(x)
#elif defined(ORC_LONG)
#define EXPS(x) expl(x)
#else
#define EXPS(x) exp(x)
#endif

/*
 * Exponential weights of one mode over one step.  With f linear on the step,
 * f(t_n + u dt) = (1-u) f^n + u f^{n+1}, the mode equation integrates exactly to
 *   f_k^{n+1} = e f_k^n + w_k dt (a0 f^n + a1 f^{n+1}),   z = lam_k dt,
 *   e = exp(-z),  a0 = int_0^1 e^{-z(1-u)} (1-u) du,  a1 = int_0^1 e^{-z(1-u)} u du.
 * With v = 1-u: a0 = int_0^1 v e^{-zv} dv = sum_j (-z)^j / (j! (j+2)) and
 * a1 = int_0^1 (1-v) e^{-zv} dv = sum_j (-z)^j / (j! (j+1) (j+2)); the series are used
 * for Re z < 1, the closed forms a0 = (1 - (1+z) e)/z^2, a1 = (z - 1 + e)/z^2 above.
 */
static void exp_weights(sc z, sc* e, sc* a0, sc* a1) {
    *e = EXPS(-z);
    if (RE(z) < 1.0) {
        sc t = 1.0, s0 = 0.0, s1 = 0.0;     /* t = (-z)^j / j! */
        for (int j = 0; j < 40; ++j) {
            s0 += t / (double)(j + 2);
            s1 += t / ((double)(j + 1) * (double)(j + 2));
            t *= -z / (double)(j + 1);
        }
        *a0 = s0;
        *a1 = s1;
    } else {
        *a0 = (1.0 - (1.0 + z) * (*e)) / (z * z);
        *a1 = (z - 1.0 + *e) / (z * z);
    }
}

/* ---- Hermite multi-index set of degrees 0 and 2 (Sec. 3.4 ordering) ---- */
typedef struct {
    int d, n;            /* space dimension, number of Hermite modes (c+1) */
    int z[MAXN][MAXD];   /* multi-indices */
} hset;

static void hset_init(hset* h, int d) {
    static const int z3[7][3] = {{0,0,0},{0,1,1},{1,0,1},{1,1,0},{0,0,2},{0,2,0},{2,0,0}};
    static const int z2[4][2] = {{0,0},{1,1},{0,2},{2,0}};
    memset(h, 0, sizeof(*h));
    h->d = d;
    if (d == 3) {
        h->n = 7;
        for (int r = 0; r < 7; ++r) for (int l = 0; l < 3; ++l) h->z[r][l] = z3[r][l];
    } else {
        h->n = 4;
        for (int r = 0; r < 4; ++r) for (int l = 0; l < 2; ++l) h->z[r][l] = z2[r][l];
    }
}

/* index of multi-index zz in the set, -1 if negative or not of degree 0/2 */
static int hset_find(const hset* h, const int* zz) {
    for (int l = 0; l < h->d; ++l) if (zz[l] < 0) return -1;
    for (int r = 0; r < h->n; ++r) {
        int same = 1;
        for (int l = 0; l < h->d; ++l) same &= (h->z[r][l] == zz[l]);
        if (same) return r;
    }
    return -1;
}

/* Coupling matrix A(kappa) (n x n, row-major): the configuration operator of
 * eq. conf_op_tested tested against psi_z / w, with a = 1/sqrt(2).
 * kap[i*d+j] = kappa_ij = d u_i / d x_j, so (grad u)_{ml} = kap[m*d+l]. */
static void build_A(const hset* h, sc De, const sc* kap, sc* A) {
    const int d = h->d, n = h->n;
    const rl a = 1 / SQRTR((rl)2);
    for (int i = 0; i < n * n; ++i) A[i] = 0.0;
    for (int r = 0; r < n; ++r) {
        const int* z = h->z[r];
        sc diag = 0.0;
        for (int l = 0; l < d; ++l) diag += (kap[l * d + l] - 1.0 / (2.0 * De)) * (double)z[l];
        A[r * n + r] += diag;
        int zz[MAXD];
        /* Phi_{(z_l - 2)} ((2a^2-1)/(2De) + kappa_ll) sqrt((z_l-1) z_l) */
        for (int l = 0; l < d; ++l) {
            if (z[l] < 2) continue;
            for (int q = 0; q < d; ++q) zz[q] = z[q];
            zz[l] -= 2;
            int col = hset_find(h, zz);
            if (col >= 0)
                A[r * n + col] += ((2.0 * a * a - 1.0) / (2.0 * De) + kap[l * d + l]) *
                                  sqrt((double)((z[l] - 1) * z[l]));
        }
        for (int l = 0; l < d; ++l) {
            for (int m = 0; m < d; ++m) {
                if (l == m) continue;
                const sc kml = kap[m * d + l];
                /* Phi_{(z_l + 1, z_m - 1)} kappa_ml sqrt((z_l+1) z_m) */
                for (int q = 0; q < d; ++q) zz[q] = z[q];
                zz[l] += 1; zz[m] -= 1;
                int col = hset_find(h, zz);
                if (col >= 0) A[r * n + col] += kml * sqrt((double)((z[l] + 1) * z[m]));
                /* Phi_{(z_l - 1, z_m - 1)} kappa_ml sqrt(z_l z_m) */
                for (int q = 0; q < d; ++q) zz[q] = z[q];
                zz[l] -= 1; zz[m] -= 1;
                col = hset_find(h, zz);
                if (col >= 0) A[r * n + col] += kml * sqrt((double)(z[l] * z[m]));
            }
        }
    }
}

/* Gaussian elimination with partial pivoting (pivot on the largest |real part|);
 * solves M x = b in place (M destroyed, b becomes x).  Returns 0 if singular. */
static int gauss_solve(int n, sc* M, sc* b) {
    for (int j = 0; j < n; ++j) {
        int p = j;
        rl best = FABSR(RE(M[j * n + j]));
        for (int i = j + 1; i < n; ++i) {
            rl v = FABSR(RE(M[i * n + j]));
            if (v > best) { best = v; p = i; }
        }
        if (best == 0.0) return 0;
        if (p != j) {
            for (int q = 0; q < n; ++q) { sc t = M[j * n + q]; M[j * n + q] = M[p * n + q]; M[p * n + q] = t; }
            sc t = b[j]; b[j] = b[p]; b[p] = t;
        }
        for (int i = j + 1; i < n; ++i) {
            sc f = M[i * n + j] / M[j * n + j];
            for (int q = j; q < n; ++q) M[i * n + q] -= f * M[j * n + q];
            b[i] -= f * b[j];
        }
    }
    for (int j = n - 1; j >= 0; --j) {
        sc s = b[j];
        for (int q = j + 1; q < n; ++q) s -= M[j * n + q] * b[q];
        b[j] = s / M[j * n + j];
    }
    return 1;
}

static void matvec(int n, const sc* A, const sc* x, sc* y) {
    for (int r = 0; r < n; ++r) {
        sc s = 0.0;
        for (int q = 0; q < n; ++q) s += A[r * n + q] * x[q];
        y[r] = s;
    }
}

/* Hermite <-> tensor map with the mass mode normalised to one (Sec. 2.1
 * definitions of the scaled Hermite functions with a = 1/sqrt(2)):
 * Phi_{2e_l} = X_ll / sqrt(2), Phi_{e_l+e_m} = X_lm, X = C - I. */
static void tensor_to_hermite(const hset* h, const sc* Xfull /* d*d */, sc mass, sc* Phi) {
    const int d = h->d;
    for (int r = 0; r < h->n; ++r) {
        const int* z = h->z[r];
        int deg = 0, i1 = -1, i2 = -1;
        for (int l = 0; l < d; ++l) {
            deg += z[l];
            for (int t = 0; t < z[l]; ++t) { if (i1 < 0) i1 = l; else i2 = l; }
        }
        if (deg == 0) Phi[r] = mass;
        else if (i1 == i2) Phi[r] = Xfull[i1 * d + i1] / SQRTR((rl)2);
        else Phi[r] = Xfull[i1 * d + i2];
    }
}

static void hermite_to_tensor(const hset* h, const sc* Phi, sc* Xfull /* d*d */) {
    const int d = h->d;
    for (int r = 0; r < h->n; ++r) {
        const int* z = h->z[r];
        int deg = 0, i1 = -1, i2 = -1;
        for (int l = 0; l < d; ++l) {
            deg += z[l];
            for (int t = 0; t < z[l]; ++t) { if (i1 < 0) i1 = l; else i2 = l; }
        }
        if (deg == 0) continue;
        if (i1 == i2) Xfull[i1 * d + i1] = SQRTR((rl)2) * Phi[r];
        else { Xfull[i1 * d + i2] = Phi[r]; Xfull[i2 * d + i1] = Phi[r]; }
    }
}

/* packed symmetric order: 2-D (xx,yy,xy), 3-D (xx,yy,zz,xy,xz,yz) */
static void packed_pair(int d, int s, int* i, int* j) {
    static const int p2[3][2] = {{0,0},{1,1},{0,1}};
    static const int p3[6][2] = {{0,0},{1,1},{2,2},{0,1},{0,2},{1,2}};
    if (d == 2) { *i = p2[s][0]; *j = p2[s][1]; }
    else { *i = p3[s][0]; *j = p3[s][1]; }
}

/* Neumaier-compensated sum of n terms x[0..n) */
static sc neumaier(int n, const sc* x) {
    sc s = 0.0, comp = 0.0;
    for (int i = 0; i < n; ++i) {
        sc t = s + x[i];
        if (FABSR(RE(s)) >= FABSR(RE(x[i]))) comp += (s - t) + x[i];
        else comp += (x[i] - t) + s;
        s = t;
    }
    return s + comp;
}

/* kappa at level lev for one point (steady when nlev == 1) */
static void kappa_level(const sc* kappa, long nlev, long npts, int d, long p, long lev, sc* out) {
    if (nlev == 1) lev = 0;
    const sc* base = kappa + (size_t)lev * d * d * npts;
    for (int q = 0; q < d * d; ++q) out[q] = base[(size_t)q * npts + p];
}

/*
 * Run nsteps time steps at every point.
 *
 * Inputs
 *   d            space dimension (2 or 3), c = d(d+1)/2 packed components
 *   npts, m      points, exponential modes (w, lam arrays of length m)
 *   De, eta_p    relaxation time and (1-beta)/Re; gamma = eta_p / De
 *   dt           time step
 *   kappa        [nlev][d*d][npts]; nlev == 1 -> steady, else nlev >= nsteps+1
 *   extrap       1: kappa at step n -> n+1 is 2 kappa^n - kappa^{n-1} (kappa^0 at n = 0);
 *                0: kappa^{n+1} (the gradient of the already updated velocity)
 *   startup      0: SDIRK2 first step; 1: BDF2 from n = 0 with a ghost level
 *                Phi^{-1} = Phi^0, Phi_k^{-1} = 0 (test mode for the convolution check);
 *                2: the exponential-mode scheme (see the header); kappa~ is then
 *                3/2 kappa^n - 1/2 kappa^{n-1} (kappa^0 at n = 0) with extrap, else kappa^{n+1}
 *   X0           [c][npts] packed initial X = C - I
 *   mass         [npts] the mass mode Phi_000 of each point, or NULL: 1 everywhere (a
 *                normalised density, Sec. 3.4).  0 gives a point without the mass mode and
 *                so without its source term: the scheme is linear in the whole vector Phi
 *                and Phi_000 is constant in time, and a coefficient of a non-constant
 *                basis function of the spatial form has no mass-mode part.
 * Outputs (any may be NULL)
 *   X_out        [2][c][npts] levels N and N-1 (N = nsteps)
 *   tau_out      [c][npts] tau^N (zero when nsteps == 0)
 *   modes_out    [2][m][c][npts] plain tensor fractional modes at levels N, N-1
 *   traj_out     [nsteps+1][c][npts] X at every level 0..N
 *   diag_out     [nsteps][6] per step: min over points of the three leading principal
 *                minors of C = I + X (2-D: the third equals the second), max ||tau||_F,
 *                sum ||tau||_F^2, count of non-finite X/tau values (real build only)
 * Returns 0 on success, 1 on bad arguments, 2 if a local system was singular.
 */
int ORC(run)(int d, long npts, int m, const sc* w, const sc* lam, sc De, sc eta_p, double dt,
             long nsteps, const sc* kappa, long nlev, int extrap, int startup, const sc* X0,
             const double* mass, sc* X_out, sc* tau_out, sc* modes_out, sc* traj_out, double* diag_out,
             int nthreads)
{
    if ((d != 2 && d != 3) || npts < 0 || m < 1 || nsteps < 0 || startup < 0 || startup > 2) return 1;
    if (nlev != 1 && nlev < nsteps + 1) return 1;
    const int c = d * (d + 1) / 2;
    hset h;
    hset_init(&h, d);
    const int n = h.n;
    const double b0 = 1.5, b1 = -2.0, b2 = 0.5;
    const rl gs = 1 - 1 / SQRTR((rl)2);   /* SDIRK2 diagonal */
    const sc gamma = eta_p / De;
    int status = 0;

#ifndef ORC_COMPLEX
    const int want_diag = diag_out != NULL;
    const int nd = 6;
    if (want_diag) {
        for (long s = 0; s < nsteps; ++s) {
            diag_out[s * nd + 0] = INFINITY; diag_out[s * nd + 1] = INFINITY; diag_out[s * nd + 2] = INFINITY;
            diag_out[s * nd + 3] = 0.0; diag_out[s * nd + 4] = 0.0; diag_out[s * nd + 5] = 0.0;
        }
    }
#endif
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif

#pragma omp parallel
    {
        /* per-thread work arrays */
        sc* Phi = (sc*)calloc(2 * n, sizeof(sc));            /* ring of 2 levels */
        sc* Phik = (sc*)calloc((size_t)2 * m * n, sizeof(sc)); /* ring of 2 levels, [lev][k][n] */
        sc* terms = (sc*)malloc(sizeof(sc) * (size_t)m);
        sc* Ek = (sc*)calloc((size_t)m * n, sizeof(sc));
        sc* Fk = (sc*)calloc((size_t)m * n, sizeof(sc));
        sc* Yk = (sc*)calloc((size_t)m * n, sizeof(sc));
#ifndef ORC_COMPLEX
        double* mydiag = want_diag ? (double*)malloc(sizeof(double) * nd * (nsteps > 0 ? nsteps : 1)) : NULL;
        if (mydiag)
            for (long s = 0; s < nsteps; ++s) {
                mydiag[s * nd + 0] = INFINITY; mydiag[s * nd + 1] = INFINITY; mydiag[s * nd + 2] = INFINITY;
                mydiag[s * nd + 3] = 0.0; mydiag[s * nd + 4] = 0.0; mydiag[s * nd + 5] = 0.0;
            }
#endif
        int mystatus = 0;

#pragma omp for schedule(static)
        for (long p = 0; p < npts; ++p) {
            sc Xf[MAXD * MAXD], kt[MAXD * MAXD], ka[MAXD * MAXD], kb[MAXD * MAXD];
            sc A[MAXN * MAXN], M[MAXN * MAXN], rhs[MAXN], v[MAXN], Av[MAXN], D[MAXN];
            /* level 0: Phi^0 = (1, Hermite image of X0), Phi_k^0 = 0 */
            for (int q = 0; q < d * d; ++q) Xf[q] = 0.0;
            for (int s = 0; s < c; ++s) {
                int i, j;
                packed_pair(d, s, &i, &j);
                Xf[i * d + j] = X0[(size_t)s * npts + p];
                Xf[j * d + i] = X0[(size_t)s * npts + p];
            }
            sc* P0 = Phi;          /* slot of level 0 */
            tensor_to_hermite(&h, Xf, mass ? (sc)mass[p] : (sc)1.0, P0);
            for (int q = 0; q < 2 * m * n; ++q) Phik[q] = 0.0;
            if (startup == 1) for (int q = 0; q < n; ++q) Phi[n + q] = P0[q]; /* ghost Phi^{-1} in slot 1 */
            if (traj_out)
                for (int s = 0; s < c; ++s) traj_out[(size_t)s * npts + p] = X0[(size_t)s * npts + p];

            for (long step = 0; step < nsteps; ++step) {
                /* velocity gradient driving step -> step+1 */
                if (extrap) {
                    /* extrapolated to t_{n+1} (BDF2 schemes) or to t_{n+1/2} (exponential) */
                    const double fa = startup == 2 ? 1.5 : 2.0, fb = startup == 2 ? -0.5 : -1.0;
                    kappa_level(kappa, nlev, npts, d, p, step, ka);
                    if (step == 0) for (int q = 0; q < d * d; ++q) kt[q] = ka[q];
                    else {
                        kappa_level(kappa, nlev, npts, d, p, step - 1, kb);
                        for (int q = 0; q < d * d; ++q) kt[q] = fa * ka[q] + fb * kb[q];
                    }
                } else {
                    kappa_level(kappa, nlev, npts, d, p, step + 1, kt);
                }
                build_A(&h, De, kt, A);
                sc* Pn = Phi + (step % 2) * n;          /* Phi^step */
                sc* Pm = Phi + ((step + 1) % 2) * n;    /* Phi^{step-1}, overwritten by Phi^{step+1} */
                sc* Kn = Phik + (size_t)(step % 2) * m * n;
                sc* Km = Phik + (size_t)((step + 1) % 2) * m * n;

                if (startup == 2) {
                    /* Phi_k^{n+1} = e_k Phi_k^n + w_k dt (a0_k Phi^n + a1_k Phi^{n+1}) and
                     * Phi^{n+1} - Phi^n = A sum_k (Phi_k^{n+1} - Phi_k^n), i.e.
                     * (I - q A) Phi^{n+1} = Phi^n + A sum_k ((e_k - 1) Phi_k^n + w_k dt a0_k Phi^n),
                     * q = sum_k w_k dt a1_k. */
                    sc q = 0.0;
                    for (int i = 0; i < n; ++i) v[i] = 0.0;
                    for (int k = 0; k < m; ++k) {
                        sc e, a0, a1;
                        exp_weights(lam[k] * dt, &e, &a0, &a1);
                        q += w[k] * dt * a1;
                        for (int i = 0; i < n; ++i) v[i] += (e - 1.0) * Kn[k * n + i] + w[k] * dt * a0 * Pn[i];
                    }
                    matvec(n, A, v, Av);
                    for (int i = 0; i < n; ++i) rhs[i] = Pn[i] + Av[i];
                    for (int i = 0; i < n * n; ++i) M[i] = -q * A[i];
                    for (int i = 0; i < n; ++i) M[i * n + i] += 1.0;
                    if (!gauss_solve(n, M, rhs)) mystatus = 2;
                    for (int k = 0; k < m; ++k) {
                        sc e, a0, a1;
                        exp_weights(lam[k] * dt, &e, &a0, &a1);
                        for (int i = 0; i < n; ++i)
                            Km[k * n + i] = e * Kn[k * n + i] + w[k] * dt * (a0 * Pn[i] + a1 * rhs[i]);
                    }
                    for (int i = 0; i < n; ++i) Pm[i] = rhs[i];
                } else if (step == 0 && startup == 0) {
                    /* SDIRK2 (Alexander) on the augmented linear system
                     *   Phi'   = A sum_k (w_k Phi - lam_k Phi_k)
                     *   Phi_k' = w_k Phi - lam_k Phi_k,  Phi_k(0) = 0.
                     * Each stage solves Y = E + h*gs*F(Y); the modes are eliminated:
                     *   Y_k = (E_k + h gs w_k Y) / (1 + h gs lam_k),
                     *   (I - h gs theta A) Y = E - h gs A sum_k lam_k E_k / (1 + h gs lam_k). */
                    const rl hg = dt * gs;
                    sc theta = 0.0;
                    for (int k = 0; k < m; ++k) theta += w[k] / (1.0 + hg * lam[k]);
                    sc Y1[MAXN], Y2[MAXN], E[MAXN], F1[MAXN];
                    for (int stage = 0; stage < 2; ++stage) {
                        if (stage == 0) {
                            for (int q = 0; q < n; ++q) E[q] = Pn[q];
                            for (int q = 0; q < m * n; ++q) Ek[q] = 0.0;
                        } else {
                            for (int q = 0; q < n; ++q) E[q] = Pn[q] + dt * (1.0 - gs) * F1[q];
                            for (int q = 0; q < m * n; ++q) Ek[q] = Kn[q] + dt * (1.0 - gs) * Fk[q];
                        }
                        for (int q = 0; q < n; ++q) {
                            sc s = 0.0;
                            for (int k = 0; k < m; ++k) s += lam[k] * Ek[k * n + q] / (1.0 + hg * lam[k]);
                            v[q] = s;
                        }
                        matvec(n, A, v, Av);
                        for (int q = 0; q < n; ++q) rhs[q] = E[q] - hg * Av[q];
                        for (int q = 0; q < n * n; ++q) M[q] = -hg * theta * A[q];
                        for (int q = 0; q < n; ++q) M[q * n + q] += 1.0;
                        if (!gauss_solve(n, M, rhs)) mystatus = 2;
                        sc* Y = stage == 0 ? Y1 : Y2;
                        for (int q = 0; q < n; ++q) Y[q] = rhs[q];
                        for (int k = 0; k < m; ++k)
                            for (int q = 0; q < n; ++q)
                                Yk[k * n + q] = (Ek[k * n + q] + hg * w[k] * Y[q]) / (1.0 + hg * lam[k]);
                        if (stage == 0) {
                            /* stage derivative F(Y1) */
                            for (int q = 0; q < n; ++q) {
                                for (int k = 0; k < m; ++k) {
                                    Fk[k * n + q] = w[k] * Y1[q] - lam[k] * Yk[k * n + q];
                                }
                            }
                            for (int q = 0; q < n; ++q) {
                                sc s = 0.0;
                                for (int k = 0; k < m; ++k) s += Fk[k * n + q];
                                v[q] = s;
                            }
                            matvec(n, A, v, F1);
                        }
                    }
                    for (int q = 0; q < n; ++q) Pm[q] = Y2[q];
                    for (int q = 0; q < m * n; ++q) Km[q] = Yk[q];
                } else {
                    /* BDF2 step, eq. FP_discrete with L = -A(kappa) (no spatial terms):
                     * (b0 I - eta A) Phi^{n+1} = -sum_j b_j (Phi^{n+1-j} - sum_k eta_k A Phi_k^{n+1-j}),
                     * eta = sum_k b0 w_k dt/(b0 + lam_k dt), eta_k = lam_k dt/(b0 + lam_k dt). */
                    sc eta = 0.0;
                    for (int k = 0; k < m; ++k) eta += b0 * w[k] * dt / (b0 + lam[k] * dt);
                    for (int q = 0; q < n; ++q) {
                        sc s = 0.0;
                        for (int k = 0; k < m; ++k) {
                            const sc etak = lam[k] * dt / (b0 + lam[k] * dt);
                            s += etak * (b1 * Kn[k * n + q] + b2 * Km[k * n + q]);
                        }
                        v[q] = s;
                    }
                    matvec(n, A, v, Av);
                    for (int q = 0; q < n; ++q) rhs[q] = -(b1 * Pn[q] + b2 * Pm[q]) + Av[q];
                    for (int q = 0; q < n * n; ++q) M[q] = -eta * A[q];
                    for (int q = 0; q < n; ++q) M[q * n + q] += b0;
                    if (!gauss_solve(n, M, rhs)) mystatus = 2;
                    /* push the modes forward, eq. BDF_Phi_k_n+1 */
                    for (int k = 0; k < m; ++k)
                        for (int q = 0; q < n; ++q)
                            Km[k * n + q] = (-(b1 * Kn[k * n + q] + b2 * Km[k * n + q]) + w[k] * dt * rhs[q]) /
                                            (b0 + lam[k] * dt);
                    for (int q = 0; q < n; ++q) Pm[q] = rhs[q];
                }

                /* kernel-compressed fractional derivative of the new level (eq.
                 * fractional_modes_fractional_derivative), Neumaier over the modes */
                sc* Pnew = Pm;
                sc* Knew = Km;
                for (int q = 0; q < n; ++q) {
                    for (int k = 0; k < m; ++k) terms[k] = w[k] * Pnew[q] - lam[k] * Knew[k * n + q];
                    D[q] = neumaier(m, terms);
                }
                const int last = (step == nsteps - 1);
                if (traj_out) {
                    sc Xn[MAXD * MAXD];
                    for (int q = 0; q < d * d; ++q) Xn[q] = 0.0;
                    hermite_to_tensor(&h, Pnew, Xn);
                    for (int s = 0; s < c; ++s) {
                        int i, j;
                        packed_pair(d, s, &i, &j);
                        traj_out[((size_t)(step + 1) * c + s) * npts + p] = Xn[i * d + j];
                    }
                }
#ifndef ORC_COMPLEX
                if (mydiag || last) {
#else
                if (last) {
#endif
                    sc Xn[MAXD * MAXD], Dt[MAXD * MAXD], tau[MAXD * MAXD];
                    for (int q = 0; q < d * d; ++q) { Xn[q] = 0.0; Dt[q] = 0.0; }
                    hermite_to_tensor(&h, Pnew, Xn);
                    hermite_to_tensor(&h, D, Dt);
                    for (int q = 0; q < d * d; ++q) tau[q] = gamma * Dt[q];
                    if (last) {
                        if (tau_out)
                            for (int s = 0; s < c; ++s) {
                                int i, j;
                                packed_pair(d, s, &i, &j);
                                tau_out[(size_t)s * npts + p] = tau[i * d + j];
                            }
                    }
#ifndef ORC_COMPLEX
                    if (mydiag) {
                        /* minima/maxima skip non-finite values (fmin/fmax); the sum of
                         * squares propagates them; entry 5 counts them */
                        double C[9], f2 = 0.0;
                        int cnt = 0;
                        for (int q = 0; q < d * d; ++q) {
                            C[q] = Xn[q] + ((q % (d + 1)) == 0 ? 1.0 : 0.0);
                            f2 += tau[q] * tau[q];
                        }
                        for (int s = 0; s < c; ++s) {
                            int i, j;
                            packed_pair(d, s, &i, &j);
                            cnt += !isfinite(Xn[i * d + j]);
                            cnt += !isfinite(tau[i * d + j]);
                        }
                        double m1 = C[0];
                        double m2 = C[0] * C[d + 1] - C[1] * C[d];
                        double m3 = m2;
                        if (d == 3)
                            m3 = C[0] * (C[4] * C[8] - C[5] * C[7]) - C[1] * (C[3] * C[8] - C[5] * C[6]) +
                                 C[2] * (C[3] * C[7] - C[4] * C[6]);
                        double* dg = mydiag + step * nd;
                        dg[0] = fmin(dg[0], m1);
                        dg[1] = fmin(dg[1], m2);
                        dg[2] = fmin(dg[2], m3);
                        dg[3] = fmax(dg[3], sqrt(f2));
                        dg[4] += f2;
                        dg[5] += (double)cnt;
                    }
#endif
                }
            }

            /* outputs: levels N and N-1 */
            const long N = nsteps;
            if (X_out) {
                for (int lv = 0; lv < 2; ++lv) {
                    long lev = N - lv;
                    sc Xn[MAXD * MAXD];
                    for (int q = 0; q < d * d; ++q) Xn[q] = 0.0;
                    if (lev >= 0) hermite_to_tensor(&h, Phi + (lev % 2) * n, Xn);
                    else for (int q = 0; q < d * d; ++q) Xn[q] = NAN;
                    for (int s = 0; s < c; ++s) {
                        int i, j;
                        packed_pair(d, s, &i, &j);
                        X_out[((size_t)lv * c + s) * npts + p] = Xn[i * d + j];
                    }
                }
            }
            if (tau_out && N == 0)
                for (int s = 0; s < c; ++s) tau_out[(size_t)s * npts + p] = 0.0;
            if (modes_out) {
                for (int lv = 0; lv < 2; ++lv) {
                    long lev = N - lv;
                    for (int k = 0; k < m; ++k) {
                        sc Xn[MAXD * MAXD];
                        for (int q = 0; q < d * d; ++q) Xn[q] = 0.0;
                        if (lev >= 0) hermite_to_tensor(&h, Phik + ((size_t)(lev % 2) * m + k) * n, Xn);
                        else for (int q = 0; q < d * d; ++q) Xn[q] = NAN;
                        for (int s = 0; s < c; ++s) {
                            int i, j;
                            packed_pair(d, s, &i, &j);
                            modes_out[(((size_t)lv * m + k) * c + s) * npts + p] = Xn[i * d + j];
                        }
                    }
                }
            }
        }

#ifndef ORC_COMPLEX
        if (mydiag) {
#pragma omp critical
            {
                for (long s = 0; s < nsteps; ++s) {
                    double* g = diag_out + s * nd;
                    const double* l = mydiag + s * nd;
                    for (int q = 0; q < 3; ++q) g[q] = fmin(g[q], l[q]);
                    g[3] = fmax(g[3], l[3]);
                    g[4] += l[4];
                    g[5] += l[5];
                }
            }
            free(mydiag);
        }
#endif
#pragma omp critical
        {
            if (mystatus) status = mystatus;
        }
        free(Phi); free(Phik); free(terms); free(Ek); free(Fk); free(Yk);
    }
    return status;
}

/* The coupling matrix for one kappa, exposed for the operator pins. */
void ORC(coupling_matrix)(int d, sc De, const sc* kap, sc* A_out) {
    hset h;
    hset_init(&h, d);
    build_A(&h, De, kap, A_out);
}

/* Hermite image (mass-normalised) of a packed tensor X, for the map pins. */
void ORC(tensor_to_hermite_packed)(int d, const sc* Xpacked, sc* Phi_out) {
    hset h;
    hset_init(&h, d);
    const int c = d * (d + 1) / 2;
    sc Xf[MAXD * MAXD];
    for (int q = 0; q < d * d; ++q) Xf[q] = 0.0;
    for (int s = 0; s < c; ++s) {
        int i, j;
        packed_pair(d, s, &i, &j);
        Xf[i * d + j] = Xpacked[s];
        Xf[j * d + i] = Xpacked[s];
    }
    tensor_to_hermite(&h, Xf, 1.0, Phi_out);
}

/* The exponential weights (e, a0, a1) of one mode at z = lam dt, for the pins. */
void ORC(exp_weights_of)(sc z, sc* out3) {
    exp_weights(z, &out3[0], &out3[1], &out3[2]);
}

/* Multi-index table of the Hermite vector (n rows of 3 ints, unused axes 0). */
int ORC(hermite_indices)(int d, int* z_out) {
    hset h;
    hset_init(&h, d);
    for (int r = 0; r < h.n; ++r)
        for (int l = 0; l < 3; ++l) z_out[r * 3 + l] = l < d ? h.z[r][l] : 0;
    return h.n;
}

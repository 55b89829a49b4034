// Stress update with the MFP equation's transport terms (advection u.grad and centre-of-mass
// diffusion eps Laplace) inside the implicit operator of the BDF2 scheme and its SDIRK2 start
// (Sec. 4.1, eq. FP_discrete), on a periodic grid with u and kappa varying in space.
//
// A step: the modes advance pointwise with the split BDF2 kernel (which also leaves each
// point's right-hand side R and history combination G), L's transport part acts on G, and
// the coupled system (a I - b K(kappa~(x)) + b T) X = rhs is solved by splitting iterations
// preconditioned by its constant-coefficient part, which is diagonal per Fourier
// coefficient.  The kernels here are single passes over the grid or the spectrum; the
// transforms are hipFFT.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

#include "tfs_device.h"
#include "tfs_internal.h"
#include "tfs_spectral.h"
#include "tfs_transport.h"

namespace tfs {
tfs_status set_error(tfs_status s, const char* msg);   // tfs_host.cpp
}

struct tfs_transport_s {
  int dim = 0, device = 0, iters = 0;
  int64_t n[3] = {1, 1, 1};
  double k0[3] = {0, 0, 0};
  double eps = 0.0;
  int64_t npoints = 0, nc = 0, stride = 0;
  hipfftHandle fwd = 0, inv = 0;     // one plane
  bool have_fwd = false, have_inv = false;
  // batched plans over c planes (forward and back) and c d planes (back), planes `stride`
  // apart on the grid; used where hipFFT takes that layout
  hipfftHandle bf = 0, bi = 0, bid = 0, bia = 0;   // bia: c (1 + d) planes (X, then grad X)
  bool batched = false;
  // grid planes: right-hand side, SDIRK2 stage-1 value, fluctuation, iterate and, right after
  // it in the same allocation, its gradients (c d planes: dg = xg + c stride)
  double *rg = nullptr, *x1g = nullptr, *fg = nullptr, *xg = nullptr, *dg = nullptr;
  // spectral planes: right-hand side, iterate, fluctuation, extra term, inverse inputs (c + c d)
  double2 *rh = nullptr, *xh = nullptr, *fh = nullptr, *eh = nullptr, *iv = nullptr;
  double *part = nullptr, *mean = nullptr;   // spatial means of kappa~ (d*d) and u~ (d)
  // GMRES (method 1): Krylov basis [iters + 1][2 c nc] doubles, dot partials, the device-side
  // state of the least-squares problem (gm_layout) and its flags (kGmFlags ints)
  int method = 0;
  double *basis = nullptr, *dpart = nullptr, *coef = nullptr;
  double* npart = nullptr;   // [kMaxBlocks] block partials of a norm taken by the update
  int* gflag = nullptr;
  hipStream_t last_stream = nullptr;   // stream of the last step (for the iteration count)
  // early exit: relative update (splitting) or residual (GMRES) below tol, tested every
  // `every` iterations (tol = 0: fixed counts; GMRES then stops at 1e-15); last_iters: the
  // most iterations one solve of the last step took
  double tol = 0.0;
  int every = 5;
  int last_iters = 0;
  double* part2 = nullptr;   // [2 kDotBlocks + 2] partials and results of the convergence test
};

namespace {

using tfs::SpecGeom;
using tfs::set_error;
using namespace tfs::dev;

constexpr int kTBlock = 256;
constexpr int kMeanBlocks = 256;

tfs_status hipfft_fail(hipfftResult r, const char* what) {
  char buf[160];
  std::snprintf(buf, sizeof(buf), "%s failed (hipfftResult %d)", what, (int)r);
  return set_error(TFS_EHIP, buf);
}

tfs_status hip_fail(hipError_t e, const char* what) {
  char buf[200];
  std::snprintf(buf, sizeof(buf), "%s: %s", what, hipGetErrorString(e));
  return set_error(TFS_EHIP, buf);
}

// The field levels of a step: kappa~ = fa ka + fb kb, u~ = fa ua + fb ub (kb, ub may be null).
struct Lev {
  const double *ka, *kb, *ua, *ub;
  double fa, fb;
};

template <int D>
__device__ __forceinline__ void level_at(const Lev& L, int64_t st, int64_t p, double (&k)[D * D], double (&u)[D]) {
#pragma unroll
  for (int q = 0; q < D * D; ++q) k[q] = L.fa * L.ka[q * st + p] + (L.kb ? L.fb * L.kb[q * st + p] : 0.0);
#pragma unroll
  for (int j = 0; j < D; ++j) u[j] = L.fa * L.ua[j * st + p] + (L.ub ? L.fb * L.ub[j * st + p] : 0.0);
}

// Block sums of kappa~ and u~ (d*d + d quantities) over a grid-stride range of points.
template <int D>
__global__ __launch_bounds__(kTBlock) void mean_partial_kernel(Lev L, int64_t npoints, int64_t st, double* part) {
  constexpr int NQ = D * D + D;
  __shared__ double red[kTBlock];
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  for (int64_t p = (int64_t)blockIdx.x * kTBlock + threadIdx.x; p < npoints; p += (int64_t)gridDim.x * kTBlock) {
    double k[D * D], u[D];
    level_at<D>(L, st, p, k, u);
#pragma unroll
    for (int q = 0; q < D * D; ++q) acc[q] += k[q];
#pragma unroll
    for (int j = 0; j < D; ++j) acc[D * D + j] += u[j];
  }
  for (int q = 0; q < NQ; ++q) {
    red[threadIdx.x] = acc[q];
    __syncthreads();
    for (int h = kTBlock / 2; h > 0; h /= 2) {
      if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
      __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x * NQ + q] = red[0];
    __syncthreads();
  }
}

__global__ void mean_finish_kernel(const double* part, int nblocks, int nq, double inv_P, double* mean) {
  const int q = threadIdx.x;
  if (q >= nq) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += part[b * nq + q];
  mean[q] = s * inv_P;
}

// SDIRK2 stage 1: R = X^0 + src1 (kappa + kappa^T).
template <int D>
__global__ __launch_bounds__(kTBlock) void start_rhs1_kernel(const double* X0, const double* ka, double src1,
                                                             int64_t npoints, int64_t st, double* R) {
  constexpr int C = Sym<D>::C;
  for (int64_t p = (int64_t)blockIdx.x * kTBlock + threadIdx.x; p < npoints; p += (int64_t)gridDim.x * kTBlock) {
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const int i = Sym<D>::i(s), j = Sym<D>::j(s);
      R[s * st + p] = X0[s * st + p] + src1 * (ka[(i * D + j) * st + p] + ka[(j * D + i) * st + p]);
    }
  }
}

// SDIRK2 stage 2, pointwise part: R = X^0 + sigma1 (K(kappa) X1 - X1/De) + sigma2 (kappa + kappa^T).
template <int D>
__global__ __launch_bounds__(kTBlock) void start_rhs2_kernel(const double* X0, const double* X1, const double* ka,
                                                             double sigma1, double sigma2, double inv_De,
                                                             int64_t npoints, int64_t st, double* R) {
  constexpr int C = Sym<D>::C;
  for (int64_t p = (int64_t)blockIdx.x * kTBlock + threadIdx.x; p < npoints; p += (int64_t)gridDim.x * kTBlock) {
    double k[D * D], x1[C], kx[C];
#pragma unroll
    for (int q = 0; q < D * D; ++q) k[q] = ka[q * st + p];
#pragma unroll
    for (int s = 0; s < C; ++s) x1[s] = X1[s * st + p];
    apply_K<D>(k, x1, kx);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const int i = Sym<D>::i(s), j = Sym<D>::j(s);
      R[s * st + p] = X0[s * st + p] + sigma1 * (kx[s] - inv_De * x1[s]) + sigma2 * (k[i * D + j] + k[j * D + i]);
    }
  }
}

// out = base + coef u~ . grad E (the gradient planes dg[(s d + j)] of the c fields E).
template <int D>
__global__ __launch_bounds__(kTBlock) void advect_add_kernel(const double* base, const double* dg, Lev L, double coef,
                                                             int64_t npoints, int64_t st, double* out) {
  constexpr int C = Sym<D>::C;
  for (int64_t p = (int64_t)blockIdx.x * kTBlock + threadIdx.x; p < npoints; p += (int64_t)gridDim.x * kTBlock) {
    double k[D * D], u[D];
    level_at<D>(L, st, p, k, u);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) a = fma(u[j], dg[(s * D + j) * st + p], a);
      out[s * st + p] = base[s * st + p] + coef * a;
    }
  }
}

// The variable part of the operator on the iterate: f = -b K(kappa~ - kappa_bar) X +
// b (u~ - u_bar) . grad X.
template <int D>
__global__ __launch_bounds__(kTBlock) void fluct_kernel(const double* X, const double* dg, Lev L, const double* mean,
                                                        double b, int64_t npoints, int64_t st, double* f) {
  constexpr int C = Sym<D>::C;
  for (int64_t p = (int64_t)blockIdx.x * kTBlock + threadIdx.x; p < npoints; p += (int64_t)gridDim.x * kTBlock) {
    double k[D * D], u[D], x[C], kx[C];
    level_at<D>(L, st, p, k, u);
#pragma unroll
    for (int q = 0; q < D * D; ++q) k[q] -= mean[q];
#pragma unroll
    for (int j = 0; j < D; ++j) u[j] -= mean[D * D + j];
#pragma unroll
    for (int s = 0; s < C; ++s) x[s] = X[s * st + p];
    apply_K<D>(k, x, kx);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) a = fma(u[j], dg[(s * D + j) * st + p], a);
      f[s * st + p] = b * (a - kx[s]);
    }
  }
}

// xi (for |xi|^2, the Nyquist wave number kept) and xd (first derivatives, Nyquist zero).
template <int D>
__device__ __forceinline__ void spec_xi(const SpecGeom& g, int64_t q, double (&xi)[D], double (&xd)[D]) {
  int64_t k[D];
  tfs::wave_numbers<D>(g, q, k);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const int64_t n = tfs::axis_n(g, j);
    const bool nyq = (n % 2 == 0) && (k[j] == n / 2 || k[j] == -n / 2);
    xi[j] = tfs::axis_k0(g, j) * (double)k[j];
    xd[j] = nyq ? 0.0 : xi[j];
  }
}

__device__ __forceinline__ double2 c_i(double s, double2 z) { return make_double2(-s * z.y, s * z.x); }

// Derivative planes i xd_j E_s at iv[(C + s D + j)] (and E itself at iv[s] when self), with
// E an unnormalised forward transform (scaled by inv_P = 1/points, so that the inverse
// transforms give grid values).
template <int D>
__global__ __launch_bounds__(kTBlock) void deriv_kernel(SpecGeom g, int64_t nc, double inv_P, const double2* E,
                                                        bool self, double2* iv) {
  constexpr int C = Sym<D>::C;
  for (int64_t q = (int64_t)blockIdx.x * kTBlock + threadIdx.x; q < nc; q += (int64_t)gridDim.x * kTBlock) {
    double xi[D], xd[D];
    spec_xi<D>(g, q, xi, xd);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      double2 e = E[s * nc + q];
      e.x *= inv_P;
      e.y *= inv_P;
      if (self) iv[s * nc + q] = e;
#pragma unroll
      for (int j = 0; j < D; ++j) iv[(C + s * D + j) * nc + q] = c_i(xd[j], e);
    }
  }
}

// rh += ae |xi|^2 E  (ae = alpha eps: the diffusion part of T applied to E, in the spectrum).
template <int D>
__global__ __launch_bounds__(kTBlock) void diffuse_add_kernel(SpecGeom g, int64_t nc, const double2* E, double ae,
                                                              double2* rh) {
  constexpr int C = Sym<D>::C;
  for (int64_t q = (int64_t)blockIdx.x * kTBlock + threadIdx.x; q < nc; q += (int64_t)gridDim.x * kTBlock) {
    double xi[D], xd[D];
    spec_xi<D>(g, q, xi, xd);
    double x2 = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) x2 = fma(xi[j], xi[j], x2);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const double2 e = E[s * nc + q];
      double2 r = rh[s * nc + q];
      r.x = fma(ae * x2, e.x, r.x);
      r.y = fma(ae * x2, e.y, r.y);
      rh[s * nc + q] = r;
    }
  }
}

// Solve (Mr + i w I) z = r for complex z (Gaussian elimination, partial pivoting by modulus).
template <int N>
__device__ __forceinline__ void solve_shifted(double (&Mr)[N][N], double w, double2 (&r)[N]) {
  double2 A[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) A[i][j] = make_double2(Mr[i][j], i == j ? w : 0.0);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    int piv = j;
    double best = A[j][j].x * A[j][j].x + A[j][j].y * A[j][j].y;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      const double v = A[i][j].x * A[i][j].x + A[i][j].y * A[i][j].y;
      if (v > best) { best = v; piv = i; }
    }
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      if (i == piv) {
#pragma unroll
        for (int t = 0; t < N; ++t) { const double2 h = A[j][t]; A[j][t] = A[i][t]; A[i][t] = h; }
        const double2 h = r[j]; r[j] = r[i]; r[i] = h;
      }
    }
    const double2 d = A[j][j];
    const double dn = 1.0 / (d.x * d.x + d.y * d.y);
    const double2 inv = make_double2(d.x * dn, -d.y * dn);
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      const double2 a = A[i][j];
      const double2 l = make_double2(a.x * inv.x - a.y * inv.y, a.x * inv.y + a.y * inv.x);
#pragma unroll
      for (int t = j + 1; t < N; ++t) {
        const double2 u = A[j][t];
        A[i][t].x -= l.x * u.x - l.y * u.y;
        A[i][t].y -= l.x * u.y + l.y * u.x;
      }
      r[i].x -= l.x * r[j].x - l.y * r[j].y;
      r[i].y -= l.x * r[j].y + l.y * r[j].x;
    }
  }
#pragma unroll
  for (int j = N - 1; j >= 0; --j) {
    double2 acc = r[j];
#pragma unroll
    for (int t = j + 1; t < N; ++t) {
      acc.x -= A[j][t].x * r[t].x - A[j][t].y * r[t].y;
      acc.y -= A[j][t].x * r[t].y + A[j][t].y * r[t].x;
    }
    const double2 d = A[j][j];
    const double dn = 1.0 / (d.x * d.x + d.y * d.y);
    r[j] = make_double2((acc.x * d.x + acc.y * d.y) * dn, (acc.y * d.x - acc.x * d.y) * dn);
  }
}

struct PrecondArgs {
  SpecGeom g;
  int64_t nc;
  double inv_P;             // rh and fh are unnormalised forward transforms
  const double2* rh;        // right-hand side coefficients [C][nc]
  const double2* fh;        // variable part's coefficients, or null
  const double* mean;       // kappa_bar (d*d), u_bar (d)
  double a, b, eps;
  double2* xh;              // new iterate [C][nc]
  double2* iv;              // inverse-transform inputs: X (C planes), i xd_j X (C D planes)
};

// X_hat = P(xi)^{-1} (rh - fh) / points, P(xi) = (a + b eps |xi|^2 + i b xd.u_bar) I - b K(kappa_bar).
template <int D>
__global__ __launch_bounds__(kTBlock) void precond_kernel(const PrecondArgs A) {
  constexpr int C = Sym<D>::C;
  double kb[D * D], ub[D];
#pragma unroll
  for (int q = 0; q < D * D; ++q) kb[q] = A.mean[q];
#pragma unroll
  for (int j = 0; j < D; ++j) ub[j] = A.mean[D * D + j];
  for (int64_t q = (int64_t)blockIdx.x * kTBlock + threadIdx.x; q < A.nc; q += (int64_t)gridDim.x * kTBlock) {
    double xi[D], xd[D];
    spec_xi<D>(A.g, q, xi, xd);
    double x2 = 0.0, xu = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      x2 = fma(xi[j], xi[j], x2);
      xu = fma(xd[j], ub[j], xu);
    }
    double2 r[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      r[s] = A.rh[s * A.nc + q];
      if (A.fh) {
        const double2 f = A.fh[s * A.nc + q];
        r[s].x -= f.x;
        r[s].y -= f.y;
      }
      r[s].x *= A.inv_P;
      r[s].y *= A.inv_P;
    }
    double M[C][C];
    build_M<D>(kb, A.a + A.b * A.eps * x2, A.b, M);
    solve_shifted<C>(M, A.b * xu, r);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      A.xh[s * A.nc + q] = r[s];
      A.iv[s * A.nc + q] = r[s];
#pragma unroll
      for (int j = 0; j < D; ++j) A.iv[(C + s * D + j) * A.nc + q] = c_i(xd[j], r[s]);
    }
  }
}

// tau = (gamma/dt) (eta X - G), G read from tau.
template <int D>
__global__ __launch_bounds__(kTBlock) void bdf2_finish_kernel(const double* X, double* tau, double eta, double ts,
                                                              int64_t npoints, int64_t st) {
  constexpr int C = Sym<D>::C;
  for (int64_t p = (int64_t)blockIdx.x * kTBlock + threadIdx.x; p < npoints; p += (int64_t)gridDim.x * kTBlock) {
#pragma unroll
    for (int s = 0; s < C; ++s) tau[s * st + p] = ts * (eta * X[s * st + p] - tau[s * st + p]);
  }
}

// SDIRK2 start, pointwise end: tau^1 = gamma (theta X2 - hr X1); modes Y_k^0 = -c_k X^0 and
// Y_k^1 = u_k X1 + v_k X2 in the plan's tiled layout.
template <int D, typename MT>
__global__ __launch_bounds__(kTBlock) void start_finish_kernel(const double* X0, const double* X1, const double* X2,
                                                               const double* coef, int m, double gamma,
                                                               double theta, double hr, double* tau, MT* Y0, MT* Y1,
                                                               int64_t npoints, int64_t st, int64_t T) {
  constexpr int C = Sym<D>::C;
  for (int64_t p = (int64_t)blockIdx.x * kTBlock + threadIdx.x; p < npoints; p += (int64_t)gridDim.x * kTBlock) {
    double x0[C], x1[C], x2[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      x0[s] = X0[s * st + p];
      x1[s] = X1[s * st + p];
      x2[s] = X2[s * st + p];
      if (tau) tau[s * st + p] = gamma * (theta * x2[s] - hr * x1[s]);
    }
    const int64_t base = (p / T) * m * C * T + p % T;
    for (int k = 0; k < m; ++k) {
      const double ck = coef[tfs::kRowC * m + k], uk = coef[tfs::kRowU * m + k], vk = coef[tfs::kRowV * m + k];
#pragma unroll
      for (int s = 0; s < C; ++s) {
        const int64_t e = base + ((int64_t)k * C + s) * T;
        Y0[e] = (MT)(-ck * x0[s]);
        Y1[e] = (MT)(uk * x1[s] + vk * x2[s]);
      }
    }
  }
}

// ---------------------------------------------------------------- GMRES on the spectrum
// Vectors are the c coefficient planes as 2 c nc doubles (re, im) with the real inner
// product: the operator is linear over the reals (the inverse transform keeps only the
// Hermitian part of a half spectrum), not over the complex numbers.
constexpr int kDotBlocks = 512;
// Most blocks of a grid-stride launch (blocks_for).
constexpr int kMaxBlocks = 256 * 16;

// part[k * kDotBlocks + b] = block b's share of <w, V_k>, k < gridDim.y (blockIdx.y = k).
// run: null, or a device flag; the launch does nothing while it is 0.
__global__ __launch_bounds__(kTBlock) void multi_dot_kernel(const double* V, int64_t nv, const double* w,
                                                            double* part, const int* run) {
  if (run && *run == 0) return;
  __shared__ double red[kTBlock];
  const double* v = V + (int64_t)blockIdx.y * nv;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kTBlock + threadIdx.x; i < nv; i += (int64_t)gridDim.x * kTBlock)
    acc = fma(w[i], v[i], acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kTBlock / 2; h > 0; h /= 2) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.y * kDotBlocks + blockIdx.x] = red[0];
}

__global__ void dot_finish_kernel(const double* part, int nvec, double* out) {
  const int k = threadIdx.x;
  if (k >= nvec) return;
  double s = 0.0;
  for (int b = 0; b < kDotBlocks; ++b) s += part[k * kDotBlocks + b];
  out[k] = s;
}

// out[k] = the kDotBlocks partials of vector k folded in a fixed order; one block per vector.
__global__ __launch_bounds__(kTBlock) void dot_fold_kernel(const double* part, double* out, const int* run) {
  if (run && *run == 0) return;
  __shared__ double red[kTBlock];
  const double* q = part + (int64_t)blockIdx.x * kDotBlocks;
  double a = 0.0;
  for (int b = threadIdx.x; b < kDotBlocks; b += kTBlock) a += q[b];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int h = kTBlock / 2; h > 0; h /= 2) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// w -= sum_k coef[k] V_k (k < nvec), or with set: w = sum_k coef[k] V_k.  nvec_dev: when not
// null the count is read from there (the device-side iteration count).
__global__ __launch_bounds__(kTBlock) void multi_axpy_kernel(const double* V, int64_t nv, int nvec,
                                                             const int* nvec_dev, const double* coef, bool set,
                                                             double* w, const int* run) {
  if (run && *run == 0) return;
  const int n = nvec_dev ? *nvec_dev : nvec;
  for (int64_t i = (int64_t)blockIdx.x * kTBlock + threadIdx.x; i < nv; i += (int64_t)gridDim.x * kTBlock) {
    double a = 0.0;
    for (int k = 0; k < n; ++k) a = fma(coef[k], V[(int64_t)k * nv + i], a);
    w[i] = set ? a : w[i] - a;
  }
}

// w -= sum_k coef[k] V_k (k < nvec), as multi_axpy_kernel, and each block's share of |w|^2
// afterwards into part[blockIdx.x] (folded by norm_fold_kernel).
__global__ __launch_bounds__(kTBlock) void axpy_norm_kernel(const double* V, int64_t nv, int nvec, const double* coef,
                                                            double* w, double* part) {
  __shared__ double red[kTBlock];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kTBlock + threadIdx.x; i < nv; i += (int64_t)gridDim.x * kTBlock) {
    double a = 0.0;
    for (int k = 0; k < nvec; ++k) a = fma(coef[k], V[(int64_t)k * nv + i], a);
    const double x = w[i] - a;
    w[i] = x;
    acc = fma(x, x, acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kTBlock / 2; h > 0; h /= 2) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out = w / sqrt(nrm2[0]), unless the flag skip is set or the norm is zero.
__global__ __launch_bounds__(kTBlock) void normalize_kernel(const double* w, int64_t nv, const double* nrm2,
                                                            const int* skip, double* out) {
  if ((skip && *skip != 0) || !(nrm2[0] > 0.0)) return;
  const double f = 1.0 / sqrt(nrm2[0]);
  for (int64_t i = (int64_t)blockIdx.x * kTBlock + threadIdx.x; i < nv; i += (int64_t)gridDim.x * kTBlock)
    out[i] = w[i] * f;
}

// ---- device-side state of GMRES's least-squares problem (no host round trip per step)
enum { kGmDone = 0, kGmK = 1, kGmReorth = 2, kGmKmax = 3, kGmFlags = 4 };

struct GmState {
  double *H, *cs, *sn, *g, *h1, *h2, *y, *nrm;   // nrm: |w'|^2, (unused), beta^2, |w_final|^2
  int* flag;
  int m;
};

// Layout of the state in one buffer of gm_doubles(m) doubles.
inline int64_t gm_doubles(int m) { return (int64_t)(m + 1) * m + 2 * m + (m + 1) + (m + 2) + (m + 1) + m + 4; }

GmState gm_layout(double* base, int* flag, int m) {
  GmState S;
  S.H = base;
  S.cs = S.H + (int64_t)(m + 1) * m;
  S.sn = S.cs + m;
  S.g = S.sn + m;
  S.h1 = S.g + (m + 1);
  S.h2 = S.h1 + (m + 2);
  S.y = S.h2 + (m + 1);
  S.nrm = S.y + m;
  S.flag = flag;
  S.m = m;
  return S;
}

// g = (beta, 0, ...); done when the right-hand side is zero (x = 0 is the solution).
__global__ void gm_start_kernel(GmState S) {
  if (threadIdx.x != 0) return;
  const double beta = sqrt(S.nrm[2]);
  for (int i = 0; i <= S.m; ++i) S.g[i] = 0.0;
  S.g[0] = beta;
  S.flag[kGmDone] = beta > 0.0 ? 0 : 1;
  S.flag[kGmK] = 0;
  S.flag[kGmReorth] = 0;
}

// |w'|^2 after the first Gram-Schmidt pass of step j (the nparts partials of
// axpy_norm_kernel folded in a fixed order) into nrm[0], and the decision on the second pass:
// it runs only where the first took off more than half of |w|^2 (h1[j + 1] holds |w|^2
// before it), the criterion of Daniel, Gragg, Kaufman and Stewart with eta = 1/sqrt(2).
__global__ __launch_bounds__(kTBlock) void norm_fold_kernel(GmState S, const double* part, int nparts, int j) {
  __shared__ double red[kTBlock];
  double a = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kTBlock) a += part[b];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int h = kTBlock / 2; h > 0; h /= 2) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    S.nrm[0] = red[0];
    S.flag[kGmReorth] = (S.flag[kGmDone] == 0 && red[0] < 0.5 * S.h1[j + 1]) ? 1 : 0;
  }
}

// Column j of the Hessenberg matrix of I + N from the projections of N v_j (one added on the
// diagonal), the earlier Givens rotations applied to it, a new rotation that zeroes its
// subdiagonal, and the residual test on g.  One wave stages the column and the rotations in
// LDS; one lane applies them (each depends on the one before).
__global__ __launch_bounds__(64) void gm_column_kernel(GmState S, int j, double tol) {
  __shared__ double col[kTBlock + 2], cs[kTBlock], sn[kTBlock];
  if (S.flag[kGmDone] != 0) return;
  const int m = S.m;
  const bool re = S.flag[kGmReorth] != 0;
  for (int i = threadIdx.x; i <= j; i += blockDim.x)
    col[i] = S.h1[i] + (re ? S.h2[i] : 0.0) + (i == j ? 1.0 : 0.0);
  for (int i = threadIdx.x; i < j; i += blockDim.x) {
    cs[i] = S.cs[i];
    sn[i] = S.sn[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double p2 = 0.0;   // |V h2|^2: what the second pass took off |w'|^2 (V orthonormal, h2 small)
    if (re)
      for (int i = 0; i <= j; ++i) p2 = fma(S.h2[i], S.h2[i], p2);
    const double n2 = S.nrm[0] - p2;
    const double hn = sqrt(n2 > 0.0 ? n2 : 0.0);
    S.nrm[3] = hn * hn;
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double a = col[i], b = col[i + 1];
      col[i] = cs[i] * a + sn[i] * b;
      col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double r = hypot(a, b);
    const double c = r > 0.0 ? a / r : 1.0, z = r > 0.0 ? b / r : 0.0;
    S.cs[j] = c;
    S.sn[j] = z;
    col[j] = r;
    col[j + 1] = 0.0;
    S.g[j + 1] = -z * S.g[j];
    S.g[j] = c * S.g[j];
    S.flag[kGmK] = j + 1;
    if (fabs(S.g[j + 1]) <= tol * sqrt(S.nrm[2]) || hn == 0.0) S.flag[kGmDone] = 1;   // |residual| / beta
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= j + 1; i += blockDim.x) S.H[(int64_t)i * m + j] = col[i];
}

// y from the k x k triangle (k = the steps taken) and g; the most steps of the step's solves.
__global__ void gm_solve_kernel(GmState S) {
  if (threadIdx.x != 0) return;
  const int m = S.m, k = S.flag[kGmK];
  for (int i = k - 1; i >= 0; --i) {
    double acc = S.g[i];
    for (int t = i + 1; t < k; ++t) acc -= S.H[(int64_t)i * m + t] * S.y[t];
    S.y[i] = acc / S.H[(int64_t)i * m + i];
  }
  if (k > S.flag[kGmKmax]) S.flag[kGmKmax] = k;
}

__global__ void gm_reset_kernel(int* flag) {
  if (threadIdx.x == 0) flag[kGmKmax] = 0;
}

// part[b] = block b's share of |x - y|^2, part[kDotBlocks + b] of |x|^2.
__global__ __launch_bounds__(kTBlock) void diff_norm_kernel(const double* x, const double* y, int64_t nv,
                                                            double* part) {
  __shared__ double r1[kTBlock], r2[kTBlock];
  double a = 0.0, b = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kTBlock + threadIdx.x; i < nv; i += (int64_t)gridDim.x * kTBlock) {
    const double d = x[i] - y[i];
    a = fma(d, d, a);
    b = fma(x[i], x[i], b);
  }
  r1[threadIdx.x] = a;
  r2[threadIdx.x] = b;
  __syncthreads();
  for (int h = kTBlock / 2; h > 0; h /= 2) {
    if ((int)threadIdx.x < h) {
      r1[threadIdx.x] += r1[threadIdx.x + h];
      r2[threadIdx.x] += r2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = r1[0];
    part[kDotBlocks + blockIdx.x] = r2[0];
  }
}

// w = P(xi)^{-1} fh / points: N v, the variable part of the preconditioned operator I + N
// applied to v (fh holds the transformed fluct(v)).
template <int D>
__global__ __launch_bounds__(kTBlock) void gm_apply_kernel(const PrecondArgs A, double2* w) {
  constexpr int C = Sym<D>::C;
  double kb[D * D], ub[D];
#pragma unroll
  for (int q = 0; q < D * D; ++q) kb[q] = A.mean[q];
#pragma unroll
  for (int j = 0; j < D; ++j) ub[j] = A.mean[D * D + j];
  for (int64_t q = (int64_t)blockIdx.x * kTBlock + threadIdx.x; q < A.nc; q += (int64_t)gridDim.x * kTBlock) {
    double xi[D], xd[D];
    spec_xi<D>(A.g, q, xi, xd);
    double x2 = 0.0, xu = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      x2 = fma(xi[j], xi[j], x2);
      xu = fma(xd[j], ub[j], xu);
    }
    double2 r[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const double2 f = A.fh[s * A.nc + q];
      r[s] = make_double2(f.x * A.inv_P, f.y * A.inv_P);
    }
    double M[C][C];
    build_M<D>(kb, A.a + A.b * A.eps * x2, A.b, M);
    solve_shifted<C>(M, A.b * xu, r);
#pragma unroll
    for (int s = 0; s < C; ++s) w[s * A.nc + q] = r[s];
  }
}

// Batched plans over c planes (forward and back) and c d planes (back), planes `stride`
// apart on the grid; s->batched tells whether hipFFT made all three.
void make_batched(tfs_transport_s* s) {
  const int dim = s->dim, c = dim * (dim + 1) / 2;
  int nn[3], eg[3], es[3];
  for (int j = 0; j < dim; ++j) nn[j] = eg[j] = es[j] = (int)s->n[j];
  es[dim - 1] = (int)(s->n[dim - 1] / 2 + 1);
  const int gd = (int)s->stride, sd = (int)s->nc;
  const bool okf = hipfftPlanMany(&s->bf, dim, nn, eg, 1, gd, es, 1, sd, HIPFFT_D2Z, c) == HIPFFT_SUCCESS;
  const bool oki = okf && hipfftPlanMany(&s->bi, dim, nn, es, 1, sd, eg, 1, gd, HIPFFT_Z2D, c) == HIPFFT_SUCCESS;
  const bool okd = oki && hipfftPlanMany(&s->bid, dim, nn, es, 1, sd, eg, 1, gd, HIPFFT_Z2D, c * dim) == HIPFFT_SUCCESS;
  const bool oka = okd && hipfftPlanMany(&s->bia, dim, nn, es, 1, sd, eg, 1, gd, HIPFFT_Z2D, c + c * dim) ==
                              HIPFFT_SUCCESS;
  s->batched = oka;
  if (!oka) {
    if (okf) hipfftDestroy(s->bf);
    if (oki) hipfftDestroy(s->bi);
    if (okd) hipfftDestroy(s->bid);
  }
}

void drop_batched(tfs_transport_s* s) {
  if (!s->batched) return;
  hipfftDestroy(s->bf);
  hipfftDestroy(s->bi);
  hipfftDestroy(s->bid);
  hipfftDestroy(s->bia);
  s->batched = false;
}

// Diagnostics of tfs.h (minors of C = I + X, max and sum of ||tau||_F^2, non-finite count):
// block partials over a grid-stride range of points, then one block folds them in order.
template <int D>
__global__ __launch_bounds__(kTBlock) void diag_partial_kernel(const double* X, const double* tau, int64_t npoints,
                                                               int64_t st, double* part) {
  constexpr int C = Sym<D>::C;
  DiagAcc acc;
  for (int64_t p = (int64_t)blockIdx.x * kTBlock + threadIdx.x; p < npoints; p += (int64_t)gridDim.x * kTBlock) {
    double x[C], t[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      x[s] = X[s * st + p];
      t[s] = tau[s * st + p];
    }
    diag_point<D>(acc, x, t);
  }
  const DiagAcc r = block_reduce(acc);
  if (threadIdx.x == 0) write_partial(part, blockIdx.x, r);
}

__global__ __launch_bounds__(kTBlock) void diag_fold_kernel(const double* part, int nparts, double* diag) {
  DiagAcc a;
  for (int i = threadIdx.x; i < nparts; i += kTBlock) {
    const double* q = part + (size_t)i * tfs::kNumDiag;
    DiagAcc b;
    b.mn1 = q[0]; b.mn2 = q[1]; b.mn3 = q[2]; b.mx = q[3]; b.sum = q[4]; b.cnt = q[5];
    diag_combine(a, b);
  }
  const DiagAcc r = block_reduce(a);
  if (threadIdx.x == 0) {
    diag[0] = r.mn1; diag[1] = r.mn2; diag[2] = r.mn3; diag[3] = r.mx; diag[4] = r.sum; diag[5] = r.cnt;
  }
}

int blocks_for(int64_t work) {
  const int64_t b = (work + kTBlock - 1) / kTBlock;
  const int64_t cap = kMaxBlocks;
  return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

SpecGeom geom(const tfs_transport_s* s) {
  SpecGeom g;
  g.n0 = s->n[0];
  g.n1 = s->n[1];
  g.n2 = s->n[2];
  g.h = s->n[s->dim - 1] / 2 + 1;
  g.k0 = s->k0[0];
  g.k1 = s->k0[1];
  g.k2 = s->k0[2];
  return g;
}

tfs_status forward_planes(tfs_transport_s* s, const double* grid, double2* spec, int count) {
  if (s->batched && count == s->dim * (s->dim + 1) / 2) {
    const hipfftResult r = hipfftExecD2Z(s->bf, const_cast<double*>(grid), (hipfftDoubleComplex*)spec);
    return r == HIPFFT_SUCCESS ? TFS_OK : hipfft_fail(r, "hipfftExecD2Z");
  }
  for (int i = 0; i < count; ++i) {
    const hipfftResult r = hipfftExecD2Z(s->fwd, const_cast<double*>(grid) + (int64_t)i * s->stride,
                                         (hipfftDoubleComplex*)(spec + (int64_t)i * s->nc));
    if (r != HIPFFT_SUCCESS) return hipfft_fail(r, "hipfftExecD2Z");
  }
  return TFS_OK;
}

tfs_status inverse_planes(tfs_transport_s* s, double2* spec, double* grid, int count) {
  const int c = s->dim * (s->dim + 1) / 2;
  if (s->batched && (count == c || count == c * s->dim || count == c + c * s->dim)) {
    const hipfftHandle h = count == c ? s->bi : (count == c * s->dim ? s->bid : s->bia);
    const hipfftResult r = hipfftExecZ2D(h, (hipfftDoubleComplex*)spec, grid);
    return r == HIPFFT_SUCCESS ? TFS_OK : hipfft_fail(r, "hipfftExecZ2D");
  }
  for (int i = 0; i < count; ++i) {
    const hipfftResult r = hipfftExecZ2D(s->inv, (hipfftDoubleComplex*)(spec + (int64_t)i * s->nc),
                                         grid + (int64_t)i * s->stride);
    if (r != HIPFFT_SUCCESS) return hipfft_fail(r, "hipfftExecZ2D");
  }
  return TFS_OK;
}

// |x - y| <= tol |x| (real inner product over nv doubles)?  Synchronises the stream.
tfs_status converged(tfs_transport_s* s, hipStream_t st, const double* x, const double* y, int64_t nv, bool* done) {
  hipLaunchKernelGGL(diff_norm_kernel, dim3(kDotBlocks), dim3(kTBlock), 0, st, x, y, nv, s->part2);
  hipLaunchKernelGGL(dot_finish_kernel, dim3(1), dim3(kTBlock), 0, st, s->part2, 2, s->part2 + 2 * kDotBlocks);
  double h[2];
  hipError_t e = hipMemcpyAsync(h, s->part2 + 2 * kDotBlocks, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "convergence test");
  *done = std::sqrt(h[0]) <= s->tol * std::sqrt(h[1]);
  return TFS_OK;
}

template <int D>
tfs_status gmres(tfs_transport_s* s, hipStream_t st, const Lev& L, const PrecondArgs& A0);

// Solve (a I - b K(kappa~) + b T) X = rhs with rhs = F^{-1}[F(rg) + alpha eps |xi|^2 E_hat]
// (E_hat = s->eh when extra), X into out.
template <int D>
tfs_status solve(tfs_transport_s* s, hipStream_t st, const Lev& L, double a, double b, bool extra, double alpha,
                 double* out) {
  constexpr int C = Sym<D>::C;
  const SpecGeom g = geom(s);
  const int bs = blocks_for(s->nc), bp = blocks_for(s->npoints);
  tfs_status r = forward_planes(s, s->rg, s->rh, C);
  if (r != TFS_OK) return r;
  if (extra) hipLaunchKernelGGL(diffuse_add_kernel<D>, dim3(bs), dim3(kTBlock), 0, st, g, s->nc, s->eh, alpha * s->eps, s->rh);
  PrecondArgs A;
  A.g = g;
  A.nc = s->nc;
  A.inv_P = 1.0 / (double)s->npoints;
  A.rh = s->rh;
  A.fh = nullptr;
  A.mean = s->mean;
  A.a = a;
  A.b = b;
  A.eps = s->eps;
  A.xh = s->xh;
  A.iv = s->iv;
  hipLaunchKernelGGL(precond_kernel<D>, dim3(bs), dim3(kTBlock), 0, st, A);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "precond_kernel launch");
  if (s->method == 1 && s->iters > 0) {
    if ((r = gmres<D>(s, st, L, A)) != TFS_OK) return r;
    return inverse_planes(s, s->iv, out, C);
  }
  A.fh = s->fh;
  const int64_t nv = (int64_t)2 * C * s->nc;
  int it = 0;
  for (; it < s->iters; ++it) {
    // the update is measured on checked iterations (s->eh is free during the iterations)
    const bool check = s->tol > 0.0 && (it + 1) % s->every == 0;
    if ((r = inverse_planes(s, s->iv, s->xg, C + C * D)) != TFS_OK) return r;    // X and grad X
    hipLaunchKernelGGL(fluct_kernel<D>, dim3(bp), dim3(kTBlock), 0, st, s->xg, s->dg, L, s->mean, b, s->npoints,
                       s->stride, s->fg);
    if ((r = forward_planes(s, s->fg, s->fh, C)) != TFS_OK) return r;
    if (check) {
      e = hipMemcpyAsync(s->eh, s->xh, sizeof(double2) * C * s->nc, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return hip_fail(e, "iterate copy");
    }
    hipLaunchKernelGGL(precond_kernel<D>, dim3(bs), dim3(kTBlock), 0, st, A);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "solver iteration launch");
    if (check) {
      bool done = false;
      if ((r = converged(s, st, reinterpret_cast<const double*>(s->xh), reinterpret_cast<const double*>(s->eh), nv,
                         &done)) != TFS_OK)
        return r;
      if (done) {
        ++it;
        break;
      }
    }
  }
  if (it > s->last_iters) s->last_iters = it;
  return inverse_planes(s, s->iv, out, C);
}

// The variable part of the operator on coefficient vector v (normalised coefficients),
// transformed: s->fh = F[fluct(F^{-1} v)] (unnormalised).
template <int D>
tfs_status apply_fluct(tfs_transport_s* s, hipStream_t st, const Lev& L, double b, const double2* v) {
  constexpr int C = Sym<D>::C;
  hipLaunchKernelGGL(deriv_kernel<D>, dim3(blocks_for(s->nc)), dim3(kTBlock), 0, st, geom(s), s->nc, 1.0, v, true,
                     s->iv);
  tfs_status r = inverse_planes(s, s->iv, s->xg, C + C * D);                     // X and grad X
  if (r != TFS_OK) return r;
  hipLaunchKernelGGL(fluct_kernel<D>, dim3(blocks_for(s->npoints)), dim3(kTBlock), 0, st, s->xg, s->dg, L, s->mean,
                     b, s->npoints, s->stride, s->fg);
  return forward_planes(s, s->fg, s->fh, C);
}

// GMRES on the preconditioned system (I + N) x = P^{-1} rhs_hat, N = P^{-1} F fluct F^{-1}
// (the splitting iteration's fixed-point equation), from x = 0, at most s->iters Arnoldi
// steps, early exit at the relative residual s->tol (1e-15 when it is 0); x into s->xh.  The
// basis is built with N, whose Krylov space is that of I + N, and the Hessenberg matrix of
// I + N is that of N with one added on the diagonal: (I + N) v_j is close to v_j where the
// splitting contracts, so orthogonalising it would cancel most of it and always call for the
// second pass, while N v_j has no such part.  Classical Gram-Schmidt, with a second pass
// where the first cancelled more than half of |w|^2.  The
// Hessenberg matrix, the Givens rotations, the residual test and the back substitution stay on
// the device, so an Arnoldi step queues its kernels without waiting; the host reads the
// residual test's flag every s->every steps to stop queueing (steps queued after convergence
// change nothing).
template <int D>
tfs_status gmres(tfs_transport_s* s, hipStream_t st, const Lev& L, const PrecondArgs& A0) {
  constexpr int C = Sym<D>::C;
  const int64_t nv = (int64_t)2 * C * s->nc;
  const int m = s->iters, bs = blocks_for(s->nc), bv = blocks_for(nv);
  double* V = s->basis;
  const GmState S = gm_layout(s->coef, s->gflag, m);
  int* done = s->gflag + kGmDone;
  int* reorth = s->gflag + kGmReorth;
  const double tol = s->tol > 0.0 ? s->tol : 1e-15;
  // b' = P^{-1} rhs_hat is in s->xh (precond_kernel); v_0 = b' / |b'|
  const double* bp = reinterpret_cast<const double*>(s->xh);
  hipLaunchKernelGGL(multi_dot_kernel, dim3(kDotBlocks, 1), dim3(kTBlock), 0, st, bp, nv, bp, s->dpart, nullptr);
  hipLaunchKernelGGL(dot_fold_kernel, dim3(1), dim3(kTBlock), 0, st, s->dpart, S.nrm + 2, nullptr);
  hipLaunchKernelGGL(gm_start_kernel, dim3(1), dim3(1), 0, st, S);
  hipLaunchKernelGGL(normalize_kernel, dim3(bv), dim3(kTBlock), 0, st, bp, nv, S.nrm + 2, done, V);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "GMRES start");
  for (int j = 0; j < m; ++j) {
    const double2* vj = reinterpret_cast<const double2*>(V + (int64_t)j * nv);
    double* w = V + (int64_t)(j + 1) * nv;             // the candidate for v_{j+1}, in its slot
    tfs_status r = apply_fluct<D>(s, st, L, A0.b, vj);
    if (r != TFS_OK) return r;
    PrecondArgs A = A0;
    A.fh = s->fh;
    hipLaunchKernelGGL(gm_apply_kernel<D>, dim3(bs), dim3(kTBlock), 0, st, A, reinterpret_cast<double2*>(w));
    // pass 1: <v_i, w> for i <= j and |w|^2 (w is vector j + 1) in one launch, then w -= V h1
    // with the partials of |w'|^2, folded with the decision on the second pass
    hipLaunchKernelGGL(multi_dot_kernel, dim3(kDotBlocks, j + 2), dim3(kTBlock), 0, st, V, nv, w, s->dpart, nullptr);
    hipLaunchKernelGGL(dot_fold_kernel, dim3(j + 2), dim3(kTBlock), 0, st, s->dpart, S.h1, nullptr);
    hipLaunchKernelGGL(axpy_norm_kernel, dim3(bv), dim3(kTBlock), 0, st, V, nv, j + 1, S.h1, w, s->npart);
    hipLaunchKernelGGL(norm_fold_kernel, dim3(1), dim3(kTBlock), 0, st, S, s->npart, bv, j);
    // pass 2 where the device decided it is needed
    hipLaunchKernelGGL(multi_dot_kernel, dim3(kDotBlocks, j + 1), dim3(kTBlock), 0, st, V, nv, w, s->dpart, reorth);
    hipLaunchKernelGGL(dot_fold_kernel, dim3(j + 1), dim3(kTBlock), 0, st, s->dpart, S.h2, reorth);
    hipLaunchKernelGGL(multi_axpy_kernel, dim3(bv), dim3(kTBlock), 0, st, V, nv, j + 1, nullptr, S.h2, false, w,
                       reorth);
    hipLaunchKernelGGL(gm_column_kernel, dim3(1), dim3(64), 0, st, S, j, tol);
    hipLaunchKernelGGL(normalize_kernel, dim3(bv), dim3(kTBlock), 0, st, w, nv, S.nrm + 3, done, w);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "GMRES step launch");
    if (j + 1 < m && (j + 1) % s->every == 0) {
      int h = 0;
      e = hipMemcpyAsync(&h, done, sizeof(int), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_fail(e, "GMRES residual test");
      if (h) break;
    }
  }
  // y from the triangle, x = V y over the steps taken (both counts read on the device)
  hipLaunchKernelGGL(gm_solve_kernel, dim3(1), dim3(1), 0, st, S);
  hipLaunchKernelGGL(multi_axpy_kernel, dim3(bv), dim3(kTBlock), 0, st, V, nv, 0, S.flag + kGmK, S.y, true,
                     reinterpret_cast<double*>(s->xh), nullptr);
  hipLaunchKernelGGL(deriv_kernel<D>, dim3(bs), dim3(kTBlock), 0, st, geom(s), s->nc, 1.0, s->xh, true, s->iv);
  e = hipGetLastError();
  return e == hipSuccess ? TFS_OK : hip_fail(e, "GMRES launch");
}

// grad of the c fields whose coefficients are in s->eh, into s->dg.
template <int D>
tfs_status gradient_of_extra(tfs_transport_s* s, hipStream_t st) {
  constexpr int C = Sym<D>::C;
  hipLaunchKernelGGL(deriv_kernel<D>, dim3(blocks_for(s->nc)), dim3(kTBlock), 0, st, geom(s), s->nc,
                     1.0 / (double)s->npoints, s->eh, false, s->iv);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "deriv_kernel launch");
  return inverse_planes(s, s->iv + (int64_t)C * s->nc, s->dg, C * D);
}

template <int D, typename MT>
tfs_status step_d(tfs_transport_s* s, const tfs_plan_s* p, int64_t n, const Lev& L, const tfs::Levels& lv,
                  double* tau, double* diag) {
  constexpr int C = Sym<D>::C;
  hipStream_t st = p->stream;
  const int bp = blocks_for(s->npoints);
  const int64_t P = s->npoints, sd = s->stride;
  hipLaunchKernelGGL(mean_partial_kernel<D>, dim3(kMeanBlocks), dim3(kTBlock), 0, st, L, P, sd, s->part);
  hipLaunchKernelGGL(mean_finish_kernel, dim3(1), dim3(64), 0, st, s->part, kMeanBlocks, D * D + D, 1.0 / (double)P,
                     s->mean);
  tfs_status r;
  if (p->scheme == TFS_SCHEME_EXP) {
    // modes, each point's R (into X^{n+1}), G (into tau) and H (into s->rg)
    hipError_t e = tfs::launch_exp_split(p, n, L.ka, L.kb, lv, tau, s->rg);
    if (e != hipSuccess) return hip_fail(e, "split step launch");
    // rhs = R + T H, then (a I - q K + q T) X = rhs with a = 1 + q/De
    if ((r = forward_planes(s, s->rg, s->eh, C)) != TFS_OK) return r;
    if ((r = gradient_of_extra<D>(s, st)) != TFS_OK) return r;
    hipLaunchKernelGGL(advect_add_kernel<D>, dim3(bp), dim3(kTBlock), 0, st, lv.Xo, s->dg, L, 1.0, P, sd, s->rg);
    if ((r = solve<D>(s, st, L, 1.0 + p->q_e / p->De, p->q_e, true, 1.0, lv.Xo)) != TFS_OK) return r;
    hipLaunchKernelGGL(bdf2_finish_kernel<D>, dim3(bp), dim3(kTBlock), 0, st, lv.Xo, tau, p->eta_e, p->tau_scale, P,
                       sd);
  } else if (n == 0) {
    const double hgt = p->hg * p->theta, inv_De = 1.0 / p->De;
    hipLaunchKernelGGL(start_rhs1_kernel<D>, dim3(bp), dim3(kTBlock), 0, st, lv.Xn, L.ka, hgt, P, sd, s->rg);
    if ((r = solve<D>(s, st, L, 1.0 + hgt * inv_De, hgt, false, 0.0, s->x1g)) != TFS_OK) return r;
    // stage 2: X^0 + sigma1 (K X1 - X1/De - T X1) + sigma2 S
    if ((r = forward_planes(s, s->x1g, s->eh, C)) != TFS_OK) return r;
    if ((r = gradient_of_extra<D>(s, st)) != TFS_OK) return r;
    hipLaunchKernelGGL(start_rhs2_kernel<D>, dim3(bp), dim3(kTBlock), 0, st, lv.Xn, s->x1g, L.ka, p->sigma1,
                       p->sigma2, inv_De, P, sd, s->rg);
    hipLaunchKernelGGL(advect_add_kernel<D>, dim3(bp), dim3(kTBlock), 0, st, s->rg, s->dg, L, -p->sigma1, P, sd,
                       s->rg);
    if ((r = solve<D>(s, st, L, 1.0 + hgt * inv_De, hgt, true, -p->sigma1, lv.Xo)) != TFS_OK) return r;
    hipLaunchKernelGGL((start_finish_kernel<D, MT>), dim3(bp), dim3(kTBlock), 0, st, lv.Xn, s->x1g, lv.Xo, p->d_coef,
                       p->m, p->gamma, p->theta, p->hr, tau, static_cast<MT*>(lv.Ym0), static_cast<MT*>(lv.Yo), P, sd,
                       p->tile);
  } else {
    // modes, each point's R (into X^{n+1}) and G (into tau)
    hipError_t e = tfs::launch_bdf2_split(p, n, L.ka, L.kb, lv, tau);
    if (e != hipSuccess) return hip_fail(e, "split step launch");
    // rhs = R + T G
    if ((r = forward_planes(s, tau, s->eh, C)) != TFS_OK) return r;
    if ((r = gradient_of_extra<D>(s, st)) != TFS_OK) return r;
    hipLaunchKernelGGL(advect_add_kernel<D>, dim3(bp), dim3(kTBlock), 0, st, lv.Xo, s->dg, L, 1.0, P, sd, s->rg);
    if ((r = solve<D>(s, st, L, p->a_diag, p->eta, true, 1.0, lv.Xo)) != TFS_OK) return r;
    hipLaunchKernelGGL(bdf2_finish_kernel<D>, dim3(bp), dim3(kTBlock), 0, st, lv.Xo, tau, p->eta, p->tau_scale, P,
                       sd);
  }
  if (diag) {   // s->part (kMeanBlocks x (d*d + d) >= kMeanBlocks x 6 doubles) is free again
    hipLaunchKernelGGL(diag_partial_kernel<D>, dim3(kMeanBlocks), dim3(kTBlock), 0, st, lv.Xo, tau, P, sd, s->part);
    hipLaunchKernelGGL(diag_fold_kernel, dim3(1), dim3(kTBlock), 0, st, s->part, kMeanBlocks, diag);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? TFS_OK : hip_fail(e, "transport step launch");
}

}  // namespace

extern "C" {

tfs_status tfs_transport_create(int dim, const int64_t* shape, const double* extent, double eps, int64_t stride,
                                int iters, tfs_transport* out) {
  if (!out) return set_error(TFS_EINVAL, "null output handle");
  *out = nullptr;
  if (dim != 2 && dim != 3) return set_error(TFS_EINVAL, "dim must be 2 or 3");
  if (!shape || !extent) return set_error(TFS_EINVAL, "null shape or extent");
  if (!(std::isfinite(eps) && eps >= 0.0)) return set_error(TFS_EINVAL, "eps must be finite and >= 0");
  if (iters < 0 || iters > 10000) return set_error(TFS_EINVAL, "iters must be in [0, 10000]");
  int64_t P = 1;
  for (int j = 0; j < dim; ++j) {
    if (shape[j] < 2 || shape[j] > (1 << 20)) return set_error(TFS_EINVAL, "every axis needs 2 .. 2^20 points");
    if (!(std::isfinite(extent[j]) && extent[j] > 0.0)) return set_error(TFS_EINVAL, "extent must be finite and > 0");
    P *= shape[j];
  }
  if (P > (int64_t)1 << 30) return set_error(TFS_EINVAL, "more than 2^30 grid points");
  if (stride < P || stride > INT32_MAX) return set_error(TFS_EINVAL, "stride must be >= the number of points and < 2^31");
  tfs_transport_s* s = new (std::nothrow) tfs_transport_s;
  if (!s) return set_error(TFS_ENOMEM, "host allocation failed");
  s->dim = dim;
  s->iters = iters;
  s->eps = eps;
  (void)hipGetDevice(&s->device);
  for (int j = 0; j < dim; ++j) {
    s->n[j] = shape[j];
    s->k0[j] = 2.0 * M_PI / extent[j];
  }
  s->npoints = P;
  s->stride = stride;
  s->nc = P / shape[dim - 1] * (shape[dim - 1] / 2 + 1);
  const int c = dim * (dim + 1) / 2, cd = c * dim;
  const size_t gp = sizeof(double) * stride, sp = sizeof(double2) * s->nc;
  hipError_t e = hipMalloc((void**)&s->rg, gp * c);
  if (e == hipSuccess) e = hipMalloc((void**)&s->x1g, gp * c);
  if (e == hipSuccess) e = hipMalloc((void**)&s->fg, gp * c);
  if (e == hipSuccess) e = hipMalloc((void**)&s->xg, gp * (c + cd));
  if (e == hipSuccess) s->dg = s->xg + (int64_t)c * stride;
  if (e == hipSuccess) e = hipMalloc((void**)&s->rh, sp * c);
  if (e == hipSuccess) e = hipMalloc((void**)&s->xh, sp * c);
  if (e == hipSuccess) e = hipMalloc((void**)&s->fh, sp * c);
  if (e == hipSuccess) e = hipMalloc((void**)&s->eh, sp * c);
  if (e == hipSuccess) e = hipMalloc((void**)&s->iv, sp * (c + cd));
  if (e == hipSuccess) e = hipMalloc((void**)&s->part, sizeof(double) * kMeanBlocks * (dim * dim + dim));
  if (e == hipSuccess) e = hipMalloc((void**)&s->mean, sizeof(double) * (dim * dim + dim));
  if (e == hipSuccess) e = hipMalloc((void**)&s->part2, sizeof(double) * (2 * kDotBlocks + 2));
  tfs_status st = TFS_OK;
  if (e != hipSuccess) st = set_error(TFS_ENOMEM, "device allocation of the transport buffers failed");
  int nn[3];
  for (int j = 0; j < dim; ++j) nn[j] = (int)shape[j];
  if (st == TFS_OK) {
    hipfftResult r = hipfftPlanMany(&s->fwd, dim, nn, nullptr, 1, 0, nullptr, 1, 0, HIPFFT_D2Z, 1);
    s->have_fwd = r == HIPFFT_SUCCESS;
    if (r == HIPFFT_SUCCESS) {
      r = hipfftPlanMany(&s->inv, dim, nn, nullptr, 1, 0, nullptr, 1, 0, HIPFFT_Z2D, 1);
      s->have_inv = r == HIPFFT_SUCCESS;
    }
    if (r != HIPFFT_SUCCESS) st = hipfft_fail(r, "hipfftPlanMany");
  }
  if (st == TFS_OK) make_batched(s);   // if hipFFT refuses the layout, single planes serve alone
  if (st != TFS_OK) {
    const std::string keep = tfs_last_error();
    tfs_transport_destroy(s);
    return set_error(st, keep.c_str());
  }
  *out = s;
  return TFS_OK;
}

tfs_status tfs_transport_destroy(tfs_transport s) {
  if (!s) return TFS_OK;
  (void)hipDeviceSynchronize();
  if (s->have_fwd) hipfftDestroy(s->fwd);
  if (s->have_inv) hipfftDestroy(s->inv);
  drop_batched(s);
  for (double* b :
       {s->rg, s->x1g, s->fg, s->xg, s->part, s->mean, s->basis, s->dpart, s->coef, s->part2, s->npart})
    if (b) (void)hipFree(b);
  if (s->gflag) (void)hipFree(s->gflag);
  for (double2* b : {s->rh, s->xh, s->fh, s->eh, s->iv})
    if (b) (void)hipFree(b);
  delete s;
  return TFS_OK;
}

int tfs_transport_batched(tfs_transport s) { return s && s->batched ? 1 : 0; }

tfs_status tfs_transport_set_tolerance(tfs_transport s, double tol, int every) {
  if (!s) return set_error(TFS_EINVAL, "null transport object");
  if (!(std::isfinite(tol) && tol >= 0.0) || every < 1) return set_error(TFS_EINVAL, "need tol >= 0 and every >= 1");
  s->tol = tol;
  s->every = every;
  return TFS_OK;
}

int tfs_transport_last_iterations(tfs_transport s) {
  if (!s) return -1;
  if (s->method != 1 || !s->gflag) return s->last_iters;
  // GMRES keeps its count on the device: read it once the last step's work is done
  int k = 0;
  hipError_t e = hipMemcpyAsync(&k, s->gflag + kGmKmax, sizeof(int), hipMemcpyDeviceToHost, s->last_stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->last_stream);
  return e == hipSuccess ? k : -1;
}

tfs_status tfs_transport_set_method(tfs_transport s, int method) {
  if (!s) return set_error(TFS_EINVAL, "null transport object");
  if (method != 0 && method != 1) return set_error(TFS_EINVAL, "method must be 0 (splitting) or 1 (GMRES)");
  if (method == 1 && s->iters > kTBlock) return set_error(TFS_EINVAL, "GMRES takes at most 256 iterations");
  if (method == 1 && !s->basis && s->iters > 0) {
    const int c = s->dim * (s->dim + 1) / 2;
    const int64_t nv = (int64_t)2 * c * s->nc;
    hipError_t e = hipMalloc((void**)&s->basis, sizeof(double) * nv * (s->iters + 1));
    if (e == hipSuccess) e = hipMalloc((void**)&s->dpart, sizeof(double) * kDotBlocks * (s->iters + 1));
    if (e == hipSuccess) e = hipMalloc((void**)&s->coef, sizeof(double) * gm_doubles(s->iters));
    if (e == hipSuccess) e = hipMalloc((void**)&s->npart, sizeof(double) * kMaxBlocks);
    if (e == hipSuccess) e = hipMalloc((void**)&s->gflag, sizeof(int) * kGmFlags);
    if (e == hipSuccess) e = hipMemset(s->gflag, 0, sizeof(int) * kGmFlags);
    if (e != hipSuccess) {
      for (double** b : {&s->basis, &s->dpart, &s->coef, &s->npart})
        if (*b) { (void)hipFree(*b); *b = nullptr; }
      if (s->gflag) { (void)hipFree(s->gflag); s->gflag = nullptr; }
      return set_error(TFS_ENOMEM, "device allocation of the Krylov basis failed");
    }
  }
  s->method = method;
  return TFS_OK;
}

tfs_status tfs_transport_set_batched(tfs_transport s, int on) {
  if (!s) return set_error(TFS_EINVAL, "null transport object");
  (void)hipDeviceSynchronize();
  if (!on) {
    drop_batched(s);
    return TFS_OK;
  }
  if (!s->batched) make_batched(s);
  return s->batched ? TFS_OK : set_error(TFS_EUNSUPPORTED, "hipFFT refuses the batched layout for this size");
}

tfs_status tfs_transport_step(tfs_transport s, tfs_plan p, int64_t n, const double* kappa_a, const double* kappa_b,
                              const double* u_a, const double* u_b, double* X, void* Y, double* tau, double* diag) {
  if (!s || !p) return set_error(TFS_EINVAL, "null transport object or plan");
  if (p->d != s->dim || p->npoints != s->npoints || p->stride != s->stride)
    return set_error(TFS_EINVAL, "plan does not match the transport object (dim, npoints, stride)");
  if (p->device != s->device) return set_error(TFS_EINVAL, "plan and transport object live on different devices");
  if (p->sp_rate || p->sp_source >= 0) return set_error(TFS_EUNSUPPORTED, "transport steps need a pointwise plan");
  if (p->kappa_f32) return set_error(TFS_EUNSUPPORTED, "transport steps take FP64 velocity gradients");
  if (p->zform) return set_error(TFS_EUNSUPPORTED, "transport steps keep the modes in the Y form (TFS_MODE_FORM_Y)");
  if (n < 0 || n >= p->max_steps) return set_error(TFS_EINVAL, "step index out of range");
  if (!kappa_a || !u_a || !X || !Y || !tau) return set_error(TFS_EINVAL, "null kappa_a, u_a, X, Y or tau");
  if (kappa_b && !u_b) return set_error(TFS_EINVAL, "u_b is needed with kappa_b");
  hipfftResult fr = hipfftSetStream(s->fwd, p->stream);
  if (fr == HIPFFT_SUCCESS) fr = hipfftSetStream(s->inv, p->stream);
  if (fr == HIPFFT_SUCCESS && s->batched) fr = hipfftSetStream(s->bf, p->stream);
  if (fr == HIPFFT_SUCCESS && s->batched) fr = hipfftSetStream(s->bi, p->stream);
  if (fr == HIPFFT_SUCCESS && s->batched) fr = hipfftSetStream(s->bid, p->stream);
  if (fr == HIPFFT_SUCCESS && s->batched) fr = hipfftSetStream(s->bia, p->stream);
  if (fr != HIPFFT_SUCCESS) return hipfft_fail(fr, "hipfftSetStream");
  Lev L;
  L.ka = kappa_a;
  L.ua = u_a;
  const bool ex = kappa_b && n >= 1;
  const bool expo = p->scheme == TFS_SCHEME_EXP;
  L.kb = ex ? kappa_b : nullptr;
  L.ub = ex ? u_b : nullptr;
  L.fa = ex ? (expo ? 1.5 : 2.0) : 1.0;      // to t_{n+1} (BDF2) or to the half step (exponential)
  L.fb = ex ? (expo ? -0.5 : -1.0) : 0.0;
  // the rings as tfs_step reads them
  const int64_t xs = (int64_t)p->c * p->stride, ys = (int64_t)p->m * p->c * p->stride;
  const size_t eb = p->precision == TFS_FP64 ? 8 : 4;
  char* Yb = static_cast<char*>(Y);
  tfs::Levels lv;
  const int sn = (int)(n % 2), sm = 1 - sn;
  if (expo) {                 // one mode level, updated in place
    lv.Xn = X + sn * xs;
    lv.Xo = X + sm * xs;
    lv.Yn = Yb;
    lv.Yo = Yb;
  } else if (n == 0) {
    lv.Xn = X;
    lv.Xo = X + xs;
    lv.Ym0 = Yb;
    lv.Yo = Yb + ys * eb;
  } else {
    lv.Xn = X + sn * xs;
    lv.Xm = X + sm * xs;
    lv.Xo = X + sm * xs;
    lv.Yn = Yb + sn * ys * eb;
    lv.Ym = Yb + sm * ys * eb;
    lv.Yo = Yb + sm * ys * eb;
  }
  s->last_iters = 0;
  s->last_stream = p->stream;
  if (s->method == 1 && s->gflag) hipLaunchKernelGGL(gm_reset_kernel, dim3(1), dim3(1), 0, p->stream, s->gflag);
  tfs_status r;
  if (p->precision == TFS_FP64)
    r = s->dim == 2 ? step_d<2, double>(s, p, n, L, lv, tau, diag) : step_d<3, double>(s, p, n, L, lv, tau, diag);
  else
    r = s->dim == 2 ? step_d<2, float>(s, p, n, L, lv, tau, diag) : step_d<3, float>(s, p, n, L, lv, tau, diag);
  if (r != TFS_OK || !(p->flags & TFS_FLAG_CHECK_SYNC)) return r;
  // as tfs_step: synchronise, and with diagnostics refuse non-finite or non-positive-definite levels
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  if (diag) {
    double h[tfs::kNumDiag];
    e = hipMemcpy(h, diag, sizeof(h), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "diagnostic read-back");
    if (h[5] != 0.0) return set_error(TFS_ENUMERIC, "non-finite entries in the new level");
    if (!(h[0] > 0.0 && h[1] > 0.0 && h[2] > 0.0))
      return set_error(TFS_ENUMERIC, "conformation not positive definite in the new level");
  }
  return TFS_OK;
}

}  // extern "C"

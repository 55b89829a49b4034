// Coupled step: pseudo-spectral projection method for the Navier-Stokes equations on a
// periodic box (Sec. 4.1, eqs. time_discretization_NS, NS_Poisson, NS_Helmholtz), coupled to
// the stress update (tfs_step with kappa^{n+1} = grad u^{n+1}).
//
// Per step: one grid kernel forms the advection (u . grad) u from the grid velocity and its
// gradient; hipFFT takes it and tau to coefficients; one spectral kernel forms the explicit
// term F = -(u.grad)u + div tau in the 2/3 band, its extrapolation, the projected Helmholtz
// solve, and the coefficients of u^{n+1} and of its d*d derivatives; hipFFT takes those back
// to the grid, where the stress update reads kappa.  Every kernel is a single pass over HBM
// (grid: 2d + d*d planes; spectrum: per coefficient the d + c transformed planes, two
// velocity levels and one explicit-term level in, one explicit-term level, one velocity
// level and d + d*d inverse-transform planes out).
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <cstdio>
#include <new>
#include <string>

#include "tfs_device.h"
#include "tfs_internal.h"
#include "tfs_ns.h"
#include "tfs_spectral.h"
#include "tfs_transport.h"

namespace tfs {
tfs_status set_error(tfs_status s, const char* msg);   // tfs_host.cpp
}

struct tfs_ns_s {
  int dim = 0;
  int device = 0;                   // the device its buffers and plans live on
  int64_t n[3] = {1, 1, 1};
  double k0[3] = {0, 0, 0};        // 2 pi / L per axis
  double nu = 0.0, dt = 0.0;
  int64_t npoints = 0, nc = 0, stride = 0;
  // Batched transforms of whole fields (d and c planes forward, d and d*d planes back), or,
  // where hipFFT refuses such a layout, one plane at a time.
  bool batched = false;
  hipfftHandle plan[4] = {0, 0, 0, 0};   // batched: fwd d, fwd c, inv d, inv d*d; else fwd, inv
  bool have[4] = {false, false, false, false};
  double* adv = nullptr;            // [d][stride] grid advection
  double2* spec_f = nullptr;        // [d + c][nc] forward transforms (advection, then tau)
  double2* spec_i = nullptr;        // [d + d*d][nc] inverse-transform inputs (u, then grad u)
  tfs_transport transport = nullptr;  // stress update with the transport terms, or null (pointwise)
};

namespace {

using tfs::set_error;

constexpr int kNsBlock = 256;

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

using tfs::SpecGeom;

// Wave vector xi of coefficient q and whether every integer wave number lies in the 2/3
// band |k_j| < n_j / 3.
template <int D>
__device__ __forceinline__ bool wave_vector(const SpecGeom& g, int64_t q, double xi[D]) {
  int64_t k[D];
  tfs::wave_numbers<D>(g, q, k);
  bool band = true;
  for (int j = 0; j < D; ++j) {
    const int64_t a = k[j] < 0 ? -k[j] : k[j];
    band = band && 3 * a < tfs::axis_n(g, j);
    xi[j] = tfs::axis_k0(g, j) * (double)k[j];
  }
  return band;
}

__device__ __forceinline__ double2 cmul_i(double s, double2 z) { return make_double2(-s * z.y, s * z.x); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 cscale(double s, double2 z) { return make_double2(s * z.x, s * z.y); }

// (u . grad) u on the grid: adv_i = sum_j u_j kappa_ij.
template <int D>
__global__ __launch_bounds__(kNsBlock) void ns_advect_kernel(const double* __restrict__ u,
                                                             const double* __restrict__ kap, double* __restrict__ adv,
                                                             int64_t npoints, int64_t stride) {
  for (int64_t p = (int64_t)blockIdx.x * kNsBlock + threadIdx.x; p < npoints; p += (int64_t)gridDim.x * kNsBlock) {
    double uu[D];
#pragma unroll
    for (int j = 0; j < D; ++j) uu[j] = u[j * stride + p];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      double s = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) s = fma(uu[j], kap[(i * D + j) * stride + p], s);
      adv[i * stride + p] = s;
    }
  }
}

struct UpdateArgs {
  SpecGeom g;
  int64_t nc;
  double inv_P;                     // transforms are unnormalised: coefficient = sum / P
  double b0dt, b1dt, b2dt;          // b_j / dt
  double a1, a2;                    // extrapolation weights
  double nu;
  const double2* fwd;               // [d + c][nc]
  const double2* uh_n;              // u^n
  const double2* uh_m;              // u^{n-1} (g = 2)
  const double2* fh_m;              // F^{n-1} (g = 2)
  double2* fh_n;                    // F^n (out)
  double2* uh_out;                  // u^{n+1} (out; may be uh_m's slot)
  double2* inv;                     // [d + d*d][nc] (out)
};

// Writes u (D planes) and i xi_j u_i (D*D planes) of one coefficient for the inverse transforms.
template <int D>
__device__ __forceinline__ void write_inverse(double2* inv, int64_t nc, int64_t q, const double xi[D],
                                              const double2 u[D]) {
#pragma unroll
  for (int i = 0; i < D; ++i) {
    inv[i * nc + q] = u[i];
#pragma unroll
    for (int j = 0; j < D; ++j) inv[(D + i * D + j) * nc + q] = cmul_i(xi[j], u[i]);
  }
}

template <int D, bool FIRST>
__global__ __launch_bounds__(kNsBlock) void ns_update_kernel(const UpdateArgs a) {
  constexpr int C = D * (D + 1) / 2;
  for (int64_t q = (int64_t)blockIdx.x * kNsBlock + threadIdx.x; q < a.nc; q += (int64_t)gridDim.x * kNsBlock) {
    double xi[D];
    const bool band = wave_vector<D>(a.g, q, xi);
    double xi2 = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) xi2 = fma(xi[j], xi[j], xi2);
    // explicit term F = -(u.grad)u + div tau, in the band
    double2 F[D];
    if (band) {
      double2 t[C];
#pragma unroll
      for (int s = 0; s < C; ++s) t[s] = cscale(a.inv_P, a.fwd[(D + s) * a.nc + q]);
#pragma unroll
      for (int i = 0; i < D; ++i) {
        double2 f = cscale(-a.inv_P, a.fwd[i * a.nc + q]);
#pragma unroll
        for (int s = 0; s < C; ++s) {
          const int si = tfs::dev::Sym<D>::i(s), sj = tfs::dev::Sym<D>::j(s);
          if (si == i) f = cadd(f, cmul_i(xi[sj], t[s]));            // d tau_{i sj} / d x_sj
          else if (sj == i) f = cadd(f, cmul_i(xi[si], t[s]));       // tau symmetric
        }
        F[i] = f;
      }
    } else {
#pragma unroll
      for (int i = 0; i < D; ++i) F[i] = make_double2(0.0, 0.0);
    }
    // R = -sum_j (b_j/dt) u^{n+1-j} + E(F)
    double2 R[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      a.fh_n[i * a.nc + q] = F[i];
      const double2 un = a.uh_n[i * a.nc + q];
      double2 r = cadd(cscale(-a.b1dt, un), cscale(a.a1, F[i]));
      if constexpr (!FIRST) {
        r = cadd(r, cscale(-a.b2dt, a.uh_m[i * a.nc + q]));
        r = cadd(r, cscale(a.a2, a.fh_m[i * a.nc + q]));
      }
      R[i] = r;
    }
    // pressure: |xi|^2 p = -i xi . R; u^{n+1} = (R - i xi p) / (b0/dt + nu |xi|^2), i.e. the
    // divergence-free part of R over the Helmholtz symbol
    double2 dot = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < D; ++j) dot = cadd(dot, cscale(xi[j], R[j]));
    const double ip = xi2 > 0.0 ? 1.0 / xi2 : 0.0;
    const double hs = 1.0 / (a.b0dt + a.nu * xi2);
    double2 un1[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double2 pr = cscale(xi[i] * ip, dot);
      un1[i] = cscale(hs, make_double2(R[i].x - pr.x, R[i].y - pr.y));
      a.uh_out[i * a.nc + q] = un1[i];
    }
    write_inverse<D>(a.inv, a.nc, q, xi, un1);
  }
}

// Level 0: the divergence-free, in-band part of a transformed grid velocity.
template <int D>
__global__ __launch_bounds__(kNsBlock) void ns_init_kernel(SpecGeom g, int64_t nc, double inv_P,
                                                           const double2* __restrict__ fwd, double2* __restrict__ uh,
                                                           double2* __restrict__ inv) {
  for (int64_t q = (int64_t)blockIdx.x * kNsBlock + threadIdx.x; q < nc; q += (int64_t)gridDim.x * kNsBlock) {
    double xi[D];
    const bool band = wave_vector<D>(g, q, xi);
    double xi2 = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) xi2 = fma(xi[j], xi[j], xi2);
    double2 u[D];
    double2 dot = make_double2(0.0, 0.0);
#pragma unroll
    for (int i = 0; i < D; ++i) {
      u[i] = band ? cscale(inv_P, fwd[i * nc + q]) : make_double2(0.0, 0.0);
      dot = cadd(dot, cscale(xi[i], u[i]));
    }
    const double ip = xi2 > 0.0 ? 1.0 / xi2 : 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      const double2 pr = cscale(xi[i] * ip, dot);
      u[i] = make_double2(u[i].x - pr.x, u[i].y - pr.y);
      uh[i * nc + q] = u[i];
    }
    write_inverse<D>(inv, nc, q, xi, u);
  }
}

int grid_blocks(int64_t work) {
  const int64_t b = (work + kNsBlock - 1) / kNsBlock;
  const int64_t cap = 256 * 16;                  // 16 blocks per compute unit
  return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

SpecGeom geom(const tfs_ns_s* s) {
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

tfs_status check_plan(const tfs_ns_s* s, const tfs_plan_s* p) {
  if (!p) return set_error(TFS_EINVAL, "null stress plan");
  if (p->d != s->dim || p->npoints != s->npoints || p->stride != s->stride)
    return set_error(TFS_EINVAL, "stress plan does not match the solver (dim, npoints, stride)");
  if (p->sp_rate || p->sp_source >= 0)
    return set_error(TFS_EINVAL, "the coupled step needs a pointwise stress plan (no spatial form set)");
  if (p->device != s->device) return set_error(TFS_EINVAL, "stress plan and solver live on different devices");
  if (!s->have[0] || !s->have[1])
    return set_error(TFS_EHIP, "the solver has no transform plans (an earlier tfs_ns_set_batched failed)");
  return TFS_OK;
}

tfs_status set_streams(tfs_ns_s* s, hipStream_t st) {
  for (int i = 0; i < 4; ++i) {
    if (!s->have[i]) continue;
    const hipfftResult r = hipfftSetStream(s->plan[i], st);
    if (r != HIPFFT_SUCCESS) return hipfft_fail(r, "hipfftSetStream");
  }
  return TFS_OK;
}

void destroy_plans(tfs_ns_s* s) {
  for (int i = 0; i < 4; ++i)
    if (s->have[i]) hipfftDestroy(s->plan[i]);
  for (int i = 0; i < 4; ++i) s->have[i] = false;
}

// batch planes of distance `stride` on the grid side and nc on the coefficient side; with
// batch = 0 one contiguous plane.
hipfftResult make_plan(tfs_ns_s* s, hipfftHandle* h, bool forward, int batch) {
  int nn[3], eg[3], es[3];
  for (int j = 0; j < s->dim; ++j) nn[j] = eg[j] = es[j] = (int)s->n[j];
  es[s->dim - 1] = (int)(s->n[s->dim - 1] / 2 + 1);
  const hipfftType t = forward ? HIPFFT_D2Z : HIPFFT_Z2D;
  if (batch == 0) return hipfftPlanMany(h, s->dim, nn, nullptr, 1, 0, nullptr, 1, 0, t, 1);
  const int gd = (int)s->stride, sd = (int)s->nc;
  return forward ? hipfftPlanMany(h, s->dim, nn, eg, 1, gd, es, 1, sd, t, batch)
                 : hipfftPlanMany(h, s->dim, nn, es, 1, sd, eg, 1, gd, t, batch);
}

tfs_status make_plans(tfs_ns_s* s, bool try_batched) {
  const int d = s->dim, c = d * (d + 1) / 2;
  const int batch[4] = {d, c, d, d * d};
  hipfftResult r = HIPFFT_SUCCESS;
  for (int i = 0; i < 4 && r == HIPFFT_SUCCESS && try_batched; ++i) {
    r = make_plan(s, &s->plan[i], i < 2, batch[i]);
    s->have[i] = r == HIPFFT_SUCCESS;
  }
  if (try_batched && r == HIPFFT_SUCCESS) {
    s->batched = true;
    return TFS_OK;
  }
  destroy_plans(s);                 // not asked for, or the batched layout was refused
  s->batched = false;
  for (int i = 0; i < 2; ++i) {
    r = make_plan(s, &s->plan[i], i == 0, 0);
    if (r != HIPFFT_SUCCESS) return hipfft_fail(r, i == 0 ? "hipfftPlanMany (D2Z)" : "hipfftPlanMany (Z2D)");
    s->have[i] = true;
  }
  return TFS_OK;
}

// Grid planes [count][stride] -> coefficient planes [count][nc]; `which` is the batched
// plan for count planes (0: d, 1: c).
tfs_status forward_planes(tfs_ns_s* s, double* grid, double2* spec, int count, int which) {
  if (s->batched) {
    const hipfftResult r = hipfftExecD2Z(s->plan[which], grid, (hipfftDoubleComplex*)spec);
    return r == HIPFFT_SUCCESS ? TFS_OK : hipfft_fail(r, "hipfftExecD2Z");
  }
  for (int i = 0; i < count; ++i) {
    const hipfftResult r = hipfftExecD2Z(s->plan[0], grid + (int64_t)i * s->stride,
                                         (hipfftDoubleComplex*)(spec + (int64_t)i * s->nc));
    if (r != HIPFFT_SUCCESS) return hipfft_fail(r, "hipfftExecD2Z");
  }
  return TFS_OK;
}

// Coefficient planes [count][nc] (overwritten) -> grid planes [count][stride]; `which` is
// the batched plan for count planes (2: d, 3: d*d).
tfs_status inverse_planes(tfs_ns_s* s, double2* spec, double* grid, int count, int which) {
  if (s->batched) {
    const hipfftResult r = hipfftExecZ2D(s->plan[which], (hipfftDoubleComplex*)spec, grid);
    return r == HIPFFT_SUCCESS ? TFS_OK : hipfft_fail(r, "hipfftExecZ2D");
  }
  for (int i = 0; i < count; ++i) {
    const hipfftResult r = hipfftExecZ2D(s->plan[1], (hipfftDoubleComplex*)(spec + (int64_t)i * s->nc),
                                         grid + (int64_t)i * s->stride);
    if (r != HIPFFT_SUCCESS) return hipfft_fail(r, "hipfftExecZ2D");
  }
  return TFS_OK;
}

template <int D>
tfs_status launch_update(const tfs_ns_s* s, hipStream_t st, int64_t n, const double2* uh_n, const double2* uh_m,
                         const double2* fh_m, double2* fh_n, double2* uh_out) {
  UpdateArgs a;
  a.g = geom(s);
  a.nc = s->nc;
  a.inv_P = 1.0 / (double)s->npoints;
  a.nu = s->nu;
  a.fwd = s->spec_f;
  a.uh_n = uh_n;
  a.uh_m = uh_m;
  a.fh_m = fh_m;
  a.fh_n = fh_n;
  a.uh_out = uh_out;
  a.inv = s->spec_i;
  const int blocks = grid_blocks(s->nc);
  if (n == 0) {                     // g = 1: BDF1, E f = f^n
    a.b0dt = 1.0 / s->dt;
    a.b1dt = -1.0 / s->dt;
    a.b2dt = 0.0;
    a.a1 = 1.0;
    a.a2 = 0.0;
    hipLaunchKernelGGL((ns_update_kernel<D, true>), dim3(blocks), dim3(kNsBlock), 0, st, a);
  } else {                          // g = 2
    a.b0dt = tfs::kB0 / s->dt;
    a.b1dt = tfs::kB1 / s->dt;
    a.b2dt = tfs::kB2 / s->dt;
    a.a1 = 2.0;
    a.a2 = -1.0;
    hipLaunchKernelGGL((ns_update_kernel<D, false>), dim3(blocks), dim3(kNsBlock), 0, st, a);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? TFS_OK : hip_fail(e, "ns_update_kernel launch");
}

}  // namespace

extern "C" {

tfs_status tfs_ns_create(int dim, const int64_t* shape, const double* extent, double nu, double dt, int64_t stride,
                         tfs_ns* out) {
  if (!out) return set_error(TFS_EINVAL, "null output handle");
  *out = nullptr;
  if (dim != 2 && dim != 3) return set_error(TFS_EINVAL, "dim must be 2 or 3");
  if (!shape || !extent) return set_error(TFS_EINVAL, "null shape or extent");
  if (!(std::isfinite(nu) && nu >= 0.0)) return set_error(TFS_EINVAL, "nu must be finite and >= 0");
  if (!(std::isfinite(dt) && dt > 0.0)) return set_error(TFS_EINVAL, "dt must be finite and > 0");
  int64_t P = 1;
  for (int j = 0; j < dim; ++j) {
    if (shape[j] < 2 || shape[j] > (1 << 20)) return set_error(TFS_EINVAL, "every axis needs 2 .. 2^20 points");
    if (!(std::isfinite(extent[j]) && extent[j] > 0.0)) return set_error(TFS_EINVAL, "extent must be finite and > 0");
    P *= shape[j];
  }
  if (P > (int64_t)1 << 30) return set_error(TFS_EINVAL, "more than 2^30 grid points");
  if (stride < P || stride > INT32_MAX) return set_error(TFS_EINVAL, "stride must be >= the number of points and < 2^31");
  tfs_ns_s* s = new (std::nothrow) tfs_ns_s;
  if (!s) return set_error(TFS_ENOMEM, "host allocation failed");
  s->dim = dim;
  (void)hipGetDevice(&s->device);
  for (int j = 0; j < dim; ++j) {
    s->n[j] = shape[j];
    s->k0[j] = 2.0 * M_PI / extent[j];
  }
  s->nu = nu;
  s->dt = dt;
  s->npoints = P;
  s->stride = stride;
  s->nc = P / shape[dim - 1] * (shape[dim - 1] / 2 + 1);
  const int c = dim * (dim + 1) / 2;
  tfs_status st = TFS_OK;
  hipError_t e = hipMalloc((void**)&s->adv, sizeof(double) * dim * stride);
  if (e == hipSuccess) e = hipMalloc((void**)&s->spec_f, sizeof(double2) * (dim + c) * s->nc);
  if (e == hipSuccess) e = hipMalloc((void**)&s->spec_i, sizeof(double2) * (dim + dim * dim) * s->nc);
  if (e != hipSuccess) st = set_error(TFS_ENOMEM, "device allocation of the solver's buffers failed");
  if (st == TFS_OK) st = make_plans(s, true);
  if (st != TFS_OK) {
    const std::string keep = tfs_last_error();
    tfs_ns_destroy(s);
    return set_error(st, keep.c_str());
  }
  *out = s;
  return TFS_OK;
}

tfs_status tfs_ns_destroy(tfs_ns s) {
  if (!s) return TFS_OK;
  (void)hipDeviceSynchronize();
  destroy_plans(s);
  if (s->adv) (void)hipFree(s->adv);
  if (s->spec_f) (void)hipFree(s->spec_f);
  if (s->spec_i) (void)hipFree(s->spec_i);
  delete s;
  return TFS_OK;
}

int64_t tfs_ns_spectral_size(tfs_ns s) { return s ? s->nc : -1; }

int tfs_ns_batched(tfs_ns s) { return s && s->batched ? 1 : 0; }

tfs_status tfs_ns_set_transport(tfs_ns s, tfs_transport tr) {
  if (!s) return set_error(TFS_EINVAL, "null solver");
  s->transport = tr;
  return TFS_OK;
}

tfs_status tfs_ns_set_batched(tfs_ns s, int on) {
  if (!s) return set_error(TFS_EINVAL, "null solver");
  (void)hipDeviceSynchronize();                 // plans of earlier launches may still run
  const tfs_status st = make_plans(s, on != 0);
  if (st != TFS_OK) return st;
  if (on && !s->batched) return set_error(TFS_EUNSUPPORTED, "hipFFT refuses the batched layout for this size");
  return TFS_OK;
}

tfs_status tfs_ns_init(tfs_ns s, tfs_plan p, double* u, void* uh, double* kappa) {
  if (!s) return set_error(TFS_EINVAL, "null solver");
  if (!u || !uh || !kappa) return set_error(TFS_EINVAL, "null u, uh or kappa");
  tfs_status st = check_plan(s, p);
  if (st != TFS_OK) return st;
  hipStream_t stream = p->stream;
  if ((st = set_streams(s, stream)) != TFS_OK) return st;
  if ((st = forward_planes(s, u, s->spec_f, s->dim, 0)) != TFS_OK) return st;
  double2* uh0 = (double2*)uh;                  // slot 0
  const int blocks = grid_blocks(s->nc);
  if (s->dim == 2)
    hipLaunchKernelGGL(ns_init_kernel<2>, dim3(blocks), dim3(kNsBlock), 0, stream, geom(s), s->nc,
                       1.0 / (double)s->npoints, s->spec_f, uh0, s->spec_i);
  else
    hipLaunchKernelGGL(ns_init_kernel<3>, dim3(blocks), dim3(kNsBlock), 0, stream, geom(s), s->nc,
                       1.0 / (double)s->npoints, s->spec_f, uh0, s->spec_i);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "ns_init_kernel launch");
  const int d = s->dim;
  if ((st = inverse_planes(s, s->spec_i, u, d, 2)) != TFS_OK) return st;
  return inverse_planes(s, s->spec_i + (int64_t)d * s->nc, kappa, d * d, 3);
}

tfs_status tfs_ns_step(tfs_ns s, tfs_plan p, int64_t n, double* u, void* uh, void* fh, double* kappa, double* X,
                       void* Y, double* tau, double* diag) {
  if (!s) return set_error(TFS_EINVAL, "null solver");
  if (!u || !uh || !fh || !kappa || !X || !Y || !tau) return set_error(TFS_EINVAL, "null field pointer");
  tfs_status st = check_plan(s, p);
  if (st != TFS_OK) return st;
  if (p->kappa_f32) return set_error(TFS_EUNSUPPORTED, "the coupled step writes FP64 velocity gradients");
  if (n < 0 || n >= p->max_steps) return set_error(TFS_EINVAL, "step index out of range");
  hipStream_t stream = p->stream;
  if ((st = set_streams(s, stream)) != TFS_OK) return st;
  const int d = s->dim;
  const int64_t lvl = (int64_t)d * s->nc;       // complex elements per ring slot
  double2* U = (double2*)uh;
  double2* Fh = (double2*)fh;
  double2* uh_n = U + (n % 2) * lvl;
  double2* uh_o = U + ((n + 1) % 2) * lvl;      // u^{n-1} in, u^{n+1} out
  double2* fh_n = Fh + (n % 2) * lvl;
  double2* fh_m = Fh + ((n + 1) % 2) * lvl;
  // advection on the grid, then the forward transforms of it and of tau
  if (d == 2)
    hipLaunchKernelGGL(ns_advect_kernel<2>, dim3(grid_blocks(s->npoints)), dim3(kNsBlock), 0, stream, u, kappa,
                       s->adv, s->npoints, s->stride);
  else
    hipLaunchKernelGGL(ns_advect_kernel<3>, dim3(grid_blocks(s->npoints)), dim3(kNsBlock), 0, stream, u, kappa,
                       s->adv, s->npoints, s->stride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "ns_advect_kernel launch");
  if ((st = forward_planes(s, s->adv, s->spec_f, d, 0)) != TFS_OK) return st;
  if ((st = forward_planes(s, tau, s->spec_f + lvl, d * (d + 1) / 2, 1)) != TFS_OK) return st;
  st = d == 2 ? launch_update<2>(s, stream, n, uh_n, uh_o, fh_m, fh_n, uh_o)
              : launch_update<3>(s, stream, n, uh_n, uh_o, fh_m, fh_n, uh_o);
  if (st != TFS_OK) return st;
  if ((st = inverse_planes(s, s->spec_i, u, d, 2)) != TFS_OK) return st;
  if ((st = inverse_planes(s, s->spec_i + lvl, kappa, d * d, 3)) != TFS_OK) return st;
  // the stress of level n+1 from kappa^{n+1} (and u^{n+1} when the transport terms are on)
  if (s->transport) return tfs_transport_step(s->transport, p, n, kappa, nullptr, u, nullptr, X, Y, tau, diag);
  return tfs_step(p, n, kappa, nullptr, X, Y, tau, diag);
}

}  // extern "C"

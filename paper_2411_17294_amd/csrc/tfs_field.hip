// Evaluation of a plan's analytic velocity gradient on its points (gfx950).
//
// The field is a sum of Fourier terms on the periodic grid [0, 2 pi)^d,
//   kappa_ij(x, t) = sum_n B_n,ij sin(k_n . x + phi_n + omega_n t),
// the same table the temporally fused launches evaluate inside their step loop.  Here it is
// written out once per time level for the step kernels: one lane per point, the phase of
// every term in FP64 and one sine each, the d*d sums in FP64, then one rounding to the
// plan's kappa precision.  About 40 FP64 operations per term and point against 4-8 bytes
// written per component: the kernel is bound by the FP64 vector units, not by HBM.
#include "tfs_device.h"
#include "tfs_internal.h"

namespace tfs {
namespace {

using namespace dev;

template <int D, typename KT>
__global__ __launch_bounds__(kBlock) void field_eval_kernel(const double* __restrict__ f, int nterms, int64_t npoints,
                                                            int64_t stride, int64_t grid, int64_t point0, double t,
                                                            const double* __restrict__ add, KT* __restrict__ out) {
  constexpr int W = D + 4 + D * D;   // k_n, phi_n, omega_n, cos/sin(omega_n dt), B_n
  const double hx = 2.0 * 3.14159265358979323846 / (double)grid;
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < npoints; p += (int64_t)gridDim.x * kBlock) {
    double x[D];
    int64_t r = point0 + p;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      x[j] = hx * (double)(r % grid);
      r /= grid;
    }
    double kap[D * D];
#pragma unroll
    for (int q = 0; q < D * D; ++q) kap[q] = 0.0;
    for (int n = 0; n < nterms; ++n) {
      const double* row = opaque_ptr(f) + n * W;
      double th = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) th += x[j] * load_uniform(row + j);
      th = th + load_uniform(row + D) + load_uniform(row + D + 1) * t;
      const double s = sin(th);
#pragma unroll
      for (int q = 0; q < D * D; ++q) kap[q] += s * load_uniform(row + D + 4 + q);
    }
#pragma unroll
    for (int q = 0; q < D * D; ++q) {
      double v = kap[q];
      if (add) v += add[q * stride + p];
      out[q * stride + p] = (KT)v;
    }
  }
}

// The lattice form of the same sum, for integer wave vectors.  On the grid k_n . x is
// (2 pi / grid) m with the integer m = sum_j k_n,j idx_j, so the term's sine is the imaginary
// part of e^{2 pi i (m mod grid) / grid} e^{i (phi_n + omega_n t)}: one lookup in the table of
// the grid's roots of unity (in LDS) and one complex product, against a sine of an FP64 phase
// per term.  It is also more accurate: the FP64 phase k . x + phi_n carries a rounding error of
// |k . x| 2^-53, the roots and the rotation a few ulp.  The rotations (cos, sin)(phi_n +
// omega_n t) are taken once per block.
template <int D, typename KT>
__global__ __launch_bounds__(kBlock) void field_lattice_kernel(const double* __restrict__ f,
                                                               const double2* __restrict__ roots_g,
                                                               const int32_t* __restrict__ kint, int nterms,
                                                               int64_t npoints, int64_t stride, int grid,
                                                               int64_t point0, double t,
                                                               const double* __restrict__ add, KT* __restrict__ out) {
  constexpr int W = D + 4 + D * D;
  extern __shared__ double2 lds[];
  double2* roots = lds;            // [grid]
  double2* rot = lds + grid;       // [nterms]
  for (int i = threadIdx.x; i < grid; i += kBlock) roots[i] = roots_g[i];
  for (int n = threadIdx.x; n < nterms; n += kBlock) {
    double sn, cn;
    sincos(f[n * W + D] + f[n * W + D + 1] * t, &sn, &cn);
    rot[n] = make_double2(cn, sn);
  }
  __syncthreads();
  const double inv_g = 1.0 / (double)grid;
  for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < npoints; p += (int64_t)gridDim.x * kBlock) {
    int idx[D];
    int64_t r = point0 + p;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      idx[j] = (int)(r % grid);
      r /= grid;
    }
    double kap[D * D];
#pragma unroll
    for (int q = 0; q < D * D; ++q) kap[q] = 0.0;
    for (int n = 0; n < nterms; ++n) {
      const int32_t* kn = opaque_ptr(kint) + n * D;
      int m = 0;
#pragma unroll
      for (int j = 0; j < D; ++j) m += load_uniform(kn + j) * idx[j];
      // m mod grid: the FP64 quotient is within one of floor(m / grid), |m| < 2^31
      int res = m - (int)floor((double)m * inv_g) * grid;
      res += res < 0 ? grid : 0;
      res -= res >= grid ? grid : 0;
      const double2 e = roots[res], ph = rot[n];
      const double s = e.y * ph.x + e.x * ph.y;     // sin(a + b)
      const double* row = opaque_ptr(f) + n * W;
#pragma unroll
      for (int q = 0; q < D * D; ++q) kap[q] += s * load_uniform(row + D + 4 + q);
    }
#pragma unroll
    for (int q = 0; q < D * D; ++q) {
      double v = kap[q];
      if (add) v += add[q * stride + p];
      out[q * stride + p] = (KT)v;
    }
  }
}

template <int D, typename KT>
hipError_t field_go(const tfs_plan_s* p, double t, const double* add, void* out) {
  int64_t g = (p->npoints + kBlock - 1) / kBlock;
  const int64_t cap = (int64_t)p->num_cus * 16;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  if (p->d_field_roots) {
    const size_t lds = sizeof(double2) * (size_t)(p->field_grid + p->field_terms);
    hipLaunchKernelGGL((field_lattice_kernel<D, KT>), dim3((unsigned)g), dim3(kBlock), lds, p->stream, p->d_field,
                       reinterpret_cast<const double2*>(p->d_field_roots), p->d_field_k, p->field_terms, p->npoints,
                       p->stride, (int)p->field_grid, p->field_point0, t, add, static_cast<KT*>(out));
  } else {
    hipLaunchKernelGGL((field_eval_kernel<D, KT>), dim3((unsigned)g), dim3(kBlock), 0, p->stream, p->d_field,
                       p->field_terms, p->npoints, p->stride, p->field_grid, p->field_point0, t, add,
                       static_cast<KT*>(out));
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_field_eval(const tfs_plan_s* p, double t, const double* add, void* out) {
  if (p->npoints == 0) return hipSuccess;
  if (p->kappa_f32) return p->d == 2 ? field_go<2, float>(p, t, add, out) : field_go<3, float>(p, t, add, out);
  return p->d == 2 ? field_go<2, double>(p, t, add, out) : field_go<3, double>(p, t, add, out);
}

}  // namespace tfs

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

template <int D, typename KT>
hipError_t field_go(const tfs_plan_s* p, double t, const double* add, void* out) {
  int64_t g = (p->npoints + kBlock - 1) / kBlock;
  const int64_t cap = (int64_t)p->num_cus * 16;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  hipLaunchKernelGGL((field_eval_kernel<D, KT>), dim3((unsigned)g), dim3(kBlock), 0, p->stream, p->d_field,
                     p->field_terms, p->npoints, p->stride, p->field_grid, p->field_point0, t, add,
                     static_cast<KT*>(out));
  return hipGetLastError();
}

}  // namespace

hipError_t launch_field_eval(const tfs_plan_s* p, double t, const double* add, void* out) {
  if (p->npoints == 0) return hipSuccess;
  if (p->kappa_f32) return p->d == 2 ? field_go<2, float>(p, t, add, out) : field_go<3, float>(p, t, add, out);
  return p->d == 2 ? field_go<2, double>(p, t, add, out) : field_go<3, double>(p, t, add, out);
}

}  // namespace tfs

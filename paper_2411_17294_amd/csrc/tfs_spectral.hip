// Fourier layout of the spatial form on a periodic box (Sec. 4.1, eq. FP_discrete with
// L = -eps Laplace - A(kappa~), diagonal where u = 0 and kappa is the same at every point).
//
// The plan's points are the real and imaginary parts of the half spectrum of hipFFT's
// real-to-complex transform, normalised so that the zero wave vector holds the mean.  One
// kernel writes the rate field eps |xi|^2 of that layout; the changes of basis are one hipFFT
// plane transform each, with a copy through the object's work buffer so that the caller's
// input stays as it was (hipFFT's complex-to-real transform overwrites its input) and the
// 1/N normalisation folded into the copy out of the forward transform.  These run before and
// after a run of steps, never inside one.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <cmath>
#include <cstdio>
#include <new>
#include <string>

#include "tfs.h"
#include "tfs_spectral.h"

namespace tfs {
tfs_status set_error(tfs_status s, const char* msg);   // tfs_host.cpp
}

struct tfs_spectral_s {
  int dim = 0;
  tfs::SpecGeom g{};
  int64_t ngrid = 0;                // N grid points
  int64_t nc = 0;                   // complex coefficients (npoints / 2)
  hipfftHandle fwd = 0, inv = 0;
  bool have_fwd = false, have_inv = false;
  double* wr = nullptr;             // [N] real plane
  double2* wc = nullptr;            // [nc] complex plane
};

namespace {

using tfs::set_error;
using tfs::SpecGeom;

constexpr int kSpecBlock = 256;
constexpr int64_t kSpecMaxBlocks = 4096;

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

unsigned blocks_for(int64_t n) {
  const int64_t b = (n + kSpecBlock - 1) / kSpecBlock;
  return (unsigned)(b < 1 ? 1 : (b > kSpecMaxBlocks ? kSpecMaxBlocks : b));
}

// rate[2q] = rate[2q + 1] = eps |xi_q|^2 for q < nc, zero on the padding up to stride.
template <int D>
__global__ __launch_bounds__(kSpecBlock) void spec_rate_kernel(SpecGeom g, int64_t nc, double eps, int64_t stride,
                                                               double* __restrict__ rate) {
  for (int64_t i = (int64_t)blockIdx.x * kSpecBlock + threadIdx.x; i < stride; i += (int64_t)gridDim.x * kSpecBlock) {
    const int64_t q = i >> 1;
    double r = 0.0;
    if (q < nc) {
      int64_t k[D];
      tfs::wave_numbers<D>(g, q, k);
      double k2 = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const double xi = (double)k[j] * tfs::axis_k0(g, j);
        k2 += xi * xi;
      }
      r = eps * k2;
    }
    rate[i] = r;
  }
}

__global__ __launch_bounds__(kSpecBlock) void spec_scale_kernel(const double* __restrict__ src, int64_t n, double s,
                                                                double* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * kSpecBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kSpecBlock)
    dst[i] = src[i] * s;
}

tfs_status set_stream(hipfftHandle h, hipStream_t st) {
  const hipfftResult r = hipfftSetStream(h, st);
  return r == HIPFFT_SUCCESS ? TFS_OK : hipfft_fail(r, "hipfftSetStream");
}

tfs_status check_planes(const tfs_spectral_s* s, const void* a, const void* b, int64_t nfields) {
  if (!s) return set_error(TFS_EINVAL, "null spectral layout");
  if (nfields < 0) return set_error(TFS_EINVAL, "nfields must be >= 0");
  if (nfields > 0 && (!a || !b)) return set_error(TFS_EINVAL, "null field buffer");
  return TFS_OK;
}

}  // namespace

extern "C" {

tfs_status tfs_spectral_create(int dim, const int64_t* shape, const double* extent, tfs_spectral* out) {
  if (!out) return set_error(TFS_EINVAL, "null output handle");
  *out = nullptr;
  if (dim != 2 && dim != 3) return set_error(TFS_EINVAL, "dim must be 2 or 3");
  if (!shape || !extent) return set_error(TFS_EINVAL, "null shape or extent");
  int64_t N = 1;
  for (int j = 0; j < dim; ++j) {
    if (shape[j] < 2 || shape[j] > (1 << 20)) return set_error(TFS_EINVAL, "every axis needs 2 .. 2^20 points");
    if (!(std::isfinite(extent[j]) && extent[j] > 0.0)) return set_error(TFS_EINVAL, "extent must be finite and > 0");
    N *= shape[j];
    if (N > (int64_t)1 << 30) return set_error(TFS_EINVAL, "more than 2^30 grid points");
  }
  tfs_spectral_s* s = new (std::nothrow) tfs_spectral_s;
  if (!s) return set_error(TFS_ENOMEM, "host allocation failed");
  s->dim = dim;
  const int64_t n[3] = {shape[0], shape[1], dim == 3 ? shape[2] : 1};
  double k0[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < dim; ++j) k0[j] = 2.0 * M_PI / extent[j];
  s->g.n0 = n[0];
  s->g.n1 = n[1];
  s->g.n2 = n[2];
  s->g.h = shape[dim - 1] / 2 + 1;
  s->g.k0 = k0[0];
  s->g.k1 = k0[1];
  s->g.k2 = k0[2];
  s->ngrid = N;
  s->nc = N / shape[dim - 1] * s->g.h;
  tfs_status st = TFS_OK;
  hipError_t e = hipMalloc((void**)&s->wr, sizeof(double) * N);
  if (e == hipSuccess) e = hipMalloc((void**)&s->wc, sizeof(double2) * s->nc);
  if (e != hipSuccess) st = set_error(TFS_ENOMEM, "device allocation of the work planes failed");
  int nn[3];
  for (int j = 0; j < dim; ++j) nn[j] = (int)shape[j];
  if (st == TFS_OK) {
    const hipfftResult r = hipfftPlanMany(&s->fwd, dim, nn, nullptr, 1, 0, nullptr, 1, 0, HIPFFT_D2Z, 1);
    s->have_fwd = r == HIPFFT_SUCCESS;
    if (!s->have_fwd) st = hipfft_fail(r, "hipfftPlanMany (D2Z)");
  }
  if (st == TFS_OK) {
    const hipfftResult r = hipfftPlanMany(&s->inv, dim, nn, nullptr, 1, 0, nullptr, 1, 0, HIPFFT_Z2D, 1);
    s->have_inv = r == HIPFFT_SUCCESS;
    if (!s->have_inv) st = hipfft_fail(r, "hipfftPlanMany (Z2D)");
  }
  if (st != TFS_OK) {
    const std::string keep = tfs_last_error();
    tfs_spectral_destroy(s);
    return set_error(st, keep.c_str());
  }
  *out = s;
  return TFS_OK;
}

tfs_status tfs_spectral_destroy(tfs_spectral s) {
  if (!s) return TFS_OK;
  (void)hipDeviceSynchronize();
  if (s->have_fwd) hipfftDestroy(s->fwd);
  if (s->have_inv) hipfftDestroy(s->inv);
  if (s->wr) (void)hipFree(s->wr);
  if (s->wc) (void)hipFree(s->wc);
  delete s;
  return TFS_OK;
}

int64_t tfs_spectral_npoints(tfs_spectral s) { return s ? 2 * s->nc : -1; }

tfs_status tfs_spectral_rate(tfs_spectral s, double eps, double* rate, int64_t stride, void* stream) {
  if (!s || !rate) return set_error(TFS_EINVAL, "null spectral layout or rate");
  if (!(std::isfinite(eps) && eps >= 0.0)) return set_error(TFS_EINVAL, "eps must be finite and >= 0");
  if (stride < 2 * s->nc) return set_error(TFS_EINVAL, "stride must be >= npoints");
  const hipStream_t st = (hipStream_t)stream;
  if (s->dim == 2)
    spec_rate_kernel<2><<<blocks_for(stride), kSpecBlock, 0, st>>>(s->g, s->nc, eps, stride, rate);
  else
    spec_rate_kernel<3><<<blocks_for(stride), kSpecBlock, 0, st>>>(s->g, s->nc, eps, stride, rate);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? TFS_OK : hip_fail(e, "spectral rate launch");
}

tfs_status tfs_spectral_to_points(tfs_spectral s, const double* grid, int64_t nfields, int64_t grid_stride,
                                  double* points, int64_t point_stride, void* stream) {
  tfs_status rc = check_planes(s, grid, points, nfields);
  if (rc != TFS_OK) return rc;
  if (grid_stride < s->ngrid || point_stride < 2 * s->nc) return set_error(TFS_EINVAL, "a plane stride is too small");
  if (nfields == 0) return TFS_OK;
  const hipStream_t st = (hipStream_t)stream;
  if ((rc = set_stream(s->fwd, st)) != TFS_OK) return rc;
  const double inv_n = 1.0 / (double)s->ngrid;
  for (int64_t f = 0; f < nfields; ++f) {
    hipError_t e = hipMemcpyAsync(s->wr, grid + f * grid_stride, sizeof(double) * s->ngrid, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "copy into the work plane");
    const hipfftResult r = hipfftExecD2Z(s->fwd, s->wr, (hipfftDoubleComplex*)s->wc);
    if (r != HIPFFT_SUCCESS) return hipfft_fail(r, "hipfftExecD2Z");
    spec_scale_kernel<<<blocks_for(2 * s->nc), kSpecBlock, 0, st>>>((const double*)s->wc, 2 * s->nc, inv_n,
                                                                     points + f * point_stride);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "spectral scale launch");
  }
  return TFS_OK;
}

tfs_status tfs_spectral_to_grid(tfs_spectral s, const double* points, int64_t nfields, int64_t point_stride,
                                double* grid, int64_t grid_stride, void* stream) {
  tfs_status rc = check_planes(s, points, grid, nfields);
  if (rc != TFS_OK) return rc;
  if (grid_stride < s->ngrid || point_stride < 2 * s->nc) return set_error(TFS_EINVAL, "a plane stride is too small");
  if (nfields == 0) return TFS_OK;
  const hipStream_t st = (hipStream_t)stream;
  if ((rc = set_stream(s->inv, st)) != TFS_OK) return rc;
  for (int64_t f = 0; f < nfields; ++f) {
    const hipError_t e = hipMemcpyAsync(s->wc, points + f * point_stride, sizeof(double2) * s->nc,
                                        hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "copy into the work plane");
    const hipfftResult r = hipfftExecZ2D(s->inv, (hipfftDoubleComplex*)s->wc, grid + f * grid_stride);
    if (r != HIPFFT_SUCCESS) return hipfft_fail(r, "hipfftExecZ2D");
  }
  return TFS_OK;
}

}  // extern "C"

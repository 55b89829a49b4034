// Index arithmetic of the half spectrum of a real periodic grid field (hipFFT's
// real-to-complex layout): coefficient q in C order over n_0 x ... x n_{d-2} x (n_{d-1}/2 + 1).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tfs {

struct SpecGeom {
  int64_t n0, n1, n2, h;            // grid sizes (unused axes 1) and the half length of the last
  double k0, k1, k2;                // 2 pi / L per axis
};

// Integer wave numbers of coefficient q: the last axis runs 0 .. n/2, the others follow the
// discrete Fourier order 0, 1, .., -1 (the Nyquist index of an even axis reads -n/2).
template <int D>
__device__ __forceinline__ void wave_numbers(const SpecGeom& g, int64_t q, int64_t (&k)[D]) {
  const int64_t nn[3] = {g.n0, g.n1, g.n2};
  int64_t idx[D];
  idx[D - 1] = q % g.h;
  int64_t rest = q / g.h;
  for (int j = D - 2; j >= 0; --j) {
    idx[j] = rest % nn[j];
    rest /= nn[j];
  }
  for (int j = 0; j < D; ++j) k[j] = (j == D - 1 || idx[j] < (nn[j] + 1) / 2) ? idx[j] : idx[j] - nn[j];
}

__host__ __device__ inline double axis_k0(const SpecGeom& g, int j) { return j == 0 ? g.k0 : (j == 1 ? g.k1 : g.k2); }
__host__ __device__ inline int64_t axis_n(const SpecGeom& g, int j) { return j == 0 ? g.n0 : (j == 1 ? g.n1 : g.n2); }

}  // namespace tfs

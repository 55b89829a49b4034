// Device helpers shared by the forward and adjoint kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "tfs_internal.h"

namespace tfs {
namespace dev {

// ------------------------------------------------------------------ packed symmetric tensors
template <int D> struct Sym;
template <> struct Sym<2> {
  static constexpr int C = 3;  // (xx, yy, xy)
  __host__ __device__ static constexpr int i(int s) { return s == 1 ? 1 : 0; }
  __host__ __device__ static constexpr int j(int s) { return s == 0 ? 0 : 1; }
};
template <> struct Sym<3> {
  static constexpr int C = 6;  // (xx, yy, zz, xy, xz, yz)
  __host__ __device__ static constexpr int i(int s) { return s < 3 ? s : (s == 5 ? 1 : 0); }
  __host__ __device__ static constexpr int j(int s) { return s < 3 ? s : (s == 3 ? 1 : 2); }
};

template <int D>
__host__ __device__ constexpr int pidx(int a, int b) {
  for (int s = 0; s < Sym<D>::C; ++s)
    if ((Sym<D>::i(s) == a && Sym<D>::j(s) == b) || (Sym<D>::i(s) == b && Sym<D>::j(s) == a)) return s;
  return -1;
}

// y = kappa x + x kappa^T on packed symmetric x.
template <int D>
__device__ __forceinline__ void apply_K(const double (&k)[D * D], const double (&x)[Sym<D>::C],
                                        double (&y)[Sym<D>::C]) {
#pragma unroll
  for (int s = 0; s < Sym<D>::C; ++s) {
    const int i = Sym<D>::i(s), j = Sym<D>::j(s);
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < D; ++l) acc += k[i * D + l] * x[pidx<D>(l, j)] + x[pidx<D>(i, l)] * k[j * D + l];
    y[s] = acc;
  }
}

// M = a I - b K(kappa), the packed matrix of X -> a X - b (kappa X + X kappa^T).
template <int D>
__device__ __forceinline__ void build_M(const double (&k)[D * D], double a, double b,
                                        double (&M)[Sym<D>::C][Sym<D>::C]) {
  constexpr int C = Sym<D>::C;
#pragma unroll
  for (int s = 0; s < C; ++s)
#pragma unroll
    for (int t = 0; t < C; ++t) M[s][t] = (s == t) ? a : 0.0;
#pragma unroll
  for (int s = 0; s < C; ++s) {
    const int i = Sym<D>::i(s), j = Sym<D>::j(s);
#pragma unroll
    for (int l = 0; l < D; ++l) {
      M[s][pidx<D>(l, j)] -= b * k[i * D + l];
      M[s][pidx<D>(i, l)] -= b * k[j * D + l];
    }
  }
}

// Solve M x = r in place (r becomes x) by Gaussian elimination with partial pivoting.
// Row exchanges are selects, so every lane runs the same instruction stream; a column's
// selects are skipped where no lane of the wave exchanges rows there (they would change
// nothing), which is the common case: the local operators are diagonally dominant at the
// workloads' time steps.
template <int N>
__device__ __forceinline__ void solve_pivot(double (&M)[N][N], double (&r)[N]) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    int p = j;
    double best = fabs(M[j][j]);
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      const double v = fabs(M[i][j]);
      const bool gt = v > best;
      best = gt ? v : best;
      p = gt ? i : p;
    }
    if (__any(p != j))
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      const bool sw = (p == i);
#pragma unroll
      for (int q = j; q < N; ++q) {
        const double t = M[j][q];
        M[j][q] = sw ? M[i][q] : t;
        M[i][q] = sw ? t : M[i][q];
      }
      const double t = r[j];
      r[j] = sw ? r[i] : t;
      r[i] = sw ? t : r[i];
    }
    const double inv = 1.0 / M[j][j];
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      const double f = M[i][j] * inv;
#pragma unroll
      for (int q = j + 1; q < N; ++q) M[i][q] -= f * M[j][q];
      r[i] -= f * r[j];
    }
  }
#pragma unroll
  for (int j = N - 1; j >= 0; --j) {
    double s = r[j];
#pragma unroll
    for (int q = j + 1; q < N; ++q) s -= M[j][q] * r[q];
    r[j] = s / M[j][j];
  }
}

// Error-free accumulation s + e += x (Knuth's TwoSum); contraction must stay off here.
__device__ __forceinline__ void two_sum_acc(double& s, double& e, double x) {
#pragma clang fp contract(off)
  const double t = s + x;
  const double bp = t - s;
  e += (s - (t - bp)) + (x - bp);
  s = t;
}

__device__ __forceinline__ double mul_rn(double a, double b) {
#pragma clang fp contract(off)
  return a * b;
}

// ------------------------------------------------------------------ wave-uniform addressing
// A wave handles 64 consecutive groups of V points.  Every access is a wave-uniform base
// (kept in scalar registers) plus a 32-bit per-lane byte offset, one per layout, instead
// of a 64-bit vector address per plane and mode.

// x is equal on all lanes; make that visible to the compiler.
__device__ __forceinline__ int64_t wave_uniform(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <typename T>
__device__ __forceinline__ const T* at(const T* base, uint32_t byte_off) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ T* at(T* base, uint32_t byte_off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off);
}

// Where a wave's points live.  Mode element (k, s) of the lane's first point is
// base + tw + (k C + s) T elements + om bytes; a plain field element is base + pw + ox bytes.
struct WaveAddr {
  int64_t pw;    // first point of the wave
  int64_t tw;    // its element offset in the tiled mode layout (tile base + offset in tile)
  uint32_t ox;   // lane's byte offset from pw in a plain FP64 field
  uint32_t om;   // lane's byte offset from tw in the mode layout
};

// Returns x unchanged, but the compiler can no longer treat it as loop-invariant: keeps
// "uniform base + per-lane offset" address sums inside a loop (one offset register)
// instead of hoisting a 64-bit per-lane address per plane out of it.
__device__ __forceinline__ uint32_t opaque(uint32_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

// The same for a wave-uniform pointer: keeps base + (k C + s) T sums inside the mode loop
// (a few scalar adds per access) instead of one hoisted scalar pair per plane.  The
// pointer passes through the asm as a global-memory pointer: a generic one would turn
// the accesses through it into flat instructions, which also count against the LDS and
// scalar-load counter, so every wait on a coefficient would wait for the data loads too.
template <typename T>
__device__ __forceinline__ T* opaque_ptr(T* p) {
  using G = __attribute__((address_space(1))) T;
  G* g = (G*)p;
  asm volatile("" : "+s"(g));
  return (T*)g;
}

// A value that every lane reads at one address, from a table no kernel of the launch
// writes (the per-mode coefficients): read through the constant address space it becomes
// a scalar load with its short latency, not a vector load that every mode waits on.
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p) {
  return *(const __attribute__((address_space(4))) T*)p;
}

// Byte offset in a plain field of element type T of the lane whose offset in an FP64 field
// is ox (the velocity gradient may be stored in FP32).
template <typename T>
__device__ __forceinline__ uint32_t field_off(uint32_t ox) {
  return sizeof(T) == 8 ? ox : ox / (uint32_t)(8 / sizeof(T));
}

// Tiled mode layout: [tile][m][c][T], point p at element (p / T) m c T + p % T of (0, 0).
template <typename MT, int C, int V>
__device__ __forceinline__ WaveAddr wave_addr(int64_t pw, int lane, int64_t T, int m) {
  WaveAddr w;
  const int64_t mcT = (int64_t)m * C * T;
  const int64_t p = pw + (int64_t)lane * V;
  w.pw = pw;
  w.tw = (pw / T) * mcT + pw % T;
  // opaque: per wave, so that no loop over waves hoists one 64-bit per-lane address per
  // field plane out of it (they would stay live across the whole kernel)
  w.ox = opaque((uint32_t)(lane * V * 8));
  w.om = (uint32_t)(((p / T) * mcT + p % T - w.tw) * (int64_t)sizeof(MT));
  return w;
}

// ------------------------------------------------------------------ vector memory access
template <typename T, int V> struct VecOf { using type = T __attribute__((ext_vector_type(V))); };
template <typename T> struct VecOf<T, 1> { using type = T; };

// NT: streaming (non-temporal) access for data touched once per step.
template <bool FULL, typename T, int V, bool NT = false>
__device__ __forceinline__ void load_v(const T* __restrict__ p, int nv, T (&o)[V]) {
  if constexpr (FULL) {
    if constexpr (V == 1) {
      o[0] = NT ? __builtin_nontemporal_load(p) : *p;
    } else {
      using vt = typename VecOf<T, V>::type;
      const vt* q = reinterpret_cast<const vt*>(p);
      const vt v = NT ? __builtin_nontemporal_load(q) : *q;
#pragma unroll
      for (int i = 0; i < V; ++i) o[i] = v[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i) {
      if (i < nv) o[i] = p[i]; else o[i] = T(0);
    }
  }
}

template <bool FULL, typename T, int V, bool NT = false>
__device__ __forceinline__ void store_v(T* p, int nv, const T (&x)[V]) {
  if constexpr (FULL) {
    if constexpr (V == 1) {
      if constexpr (NT) __builtin_nontemporal_store(x[0], p); else *p = x[0];
    } else {
      using vt = typename VecOf<T, V>::type;
      vt v;
#pragma unroll
      for (int i = 0; i < V; ++i) v[i] = x[i];
      if constexpr (NT) __builtin_nontemporal_store(v, reinterpret_cast<vt*>(p));
      else *reinterpret_cast<vt*>(p) = v;
    }
  } else {
#pragma unroll
    for (int i = 0; i < V; ++i)
      if (i < nv) p[i] = x[i];
  }
}

// ------------------------------------------------------------------ diagnostics
struct DiagAcc {
  double mn1 = INFINITY, mn2 = INFINITY, mn3 = INFINITY, mx = 0.0, sum = 0.0, cnt = 0.0;
};

template <int D>
__device__ __forceinline__ void diag_point(DiagAcc& a, const double (&x)[Sym<D>::C], const double (&t)[Sym<D>::C]) {
  constexpr int C = Sym<D>::C;
  double f2 = 0.0, cnt = 0.0;
#pragma unroll
  for (int s = 0; s < C; ++s) {
    const double w = (s < D) ? 1.0 : 2.0;  // off-diagonal entries appear twice in the full tensor
    f2 += w * t[s] * t[s];
    cnt += (isfinite(x[s]) ? 0.0 : 1.0) + (isfinite(t[s]) ? 0.0 : 1.0);
  }
  double m1, m2, m3;
  if constexpr (D == 2) {
    const double cxx = 1.0 + x[0], cyy = 1.0 + x[1], cxy = x[2];
    m1 = cxx;
    m2 = cxx * cyy - cxy * cxy;
    m3 = m2;
  } else {
    const double a00 = 1.0 + x[0], a11 = 1.0 + x[1], a22 = 1.0 + x[2];
    const double a01 = x[3], a02 = x[4], a12 = x[5];
    m1 = a00;
    m2 = a00 * a11 - a01 * a01;
    m3 = a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) + a02 * (a01 * a12 - a11 * a02);
  }
  a.mn1 = fmin(a.mn1, m1);
  a.mn2 = fmin(a.mn2, m2);
  a.mn3 = fmin(a.mn3, m3);
  a.mx = fmax(a.mx, sqrt(f2));
  a.sum += f2;
  a.cnt += cnt;
}

__device__ __forceinline__ void diag_combine(DiagAcc& a, const DiagAcc& b) {
  a.mn1 = fmin(a.mn1, b.mn1);
  a.mn2 = fmin(a.mn2, b.mn2);
  a.mn3 = fmin(a.mn3, b.mn3);
  a.mx = fmax(a.mx, b.mx);
  a.sum += b.sum;
  a.cnt += b.cnt;
}

// Deterministic block reduction: butterfly within each 64-lane wave, then the waves in
// order through LDS; thread 0 returns the block total.
__device__ inline DiagAcc block_reduce(DiagAcc a) {
  __shared__ double sh[kBlock / 64][kNumDiag];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    DiagAcc b;
    b.mn1 = __shfl_xor(a.mn1, off);
    b.mn2 = __shfl_xor(a.mn2, off);
    b.mn3 = __shfl_xor(a.mn3, off);
    b.mx = __shfl_xor(a.mx, off);
    b.sum = __shfl_xor(a.sum, off);
    b.cnt = __shfl_xor(a.cnt, off);
    diag_combine(a, b);
  }
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) {
    sh[wave][0] = a.mn1; sh[wave][1] = a.mn2; sh[wave][2] = a.mn3;
    sh[wave][3] = a.mx; sh[wave][4] = a.sum; sh[wave][5] = a.cnt;
  }
  __syncthreads();
  DiagAcc r;
  if (threadIdx.x == 0) {
    for (int w = 0; w < kBlock / 64; ++w) {
      DiagAcc b;
      b.mn1 = sh[w][0]; b.mn2 = sh[w][1]; b.mn3 = sh[w][2];
      b.mx = sh[w][3]; b.sum = sh[w][4]; b.cnt = sh[w][5];
      diag_combine(r, b);
    }
  }
  return r;
}

__device__ __forceinline__ void write_partial(double* part, int slot, const DiagAcc& r) {
  double* o = part + (size_t)slot * kNumDiag;
  o[0] = r.mn1; o[1] = r.mn2; o[2] = r.mn3; o[3] = r.mx; o[4] = r.sum; o[5] = r.cnt;
}


}  // namespace dev
}  // namespace tfs

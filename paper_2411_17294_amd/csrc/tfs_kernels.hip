// HIP kernels (gfx950) of the time-fractional extra-stress update.
//
// One lane owns V consecutive points of the structure-of-arrays fields and runs the
// whole step for them in registers:
//   * BDF2 step (Sec. 4.1, eqs. BDF_Phi_k_n+1 and FP_discrete, pointwise in tensor
//     variables with the mode representation Y_k = X_k - c_k X):
//       P        = 2 X^n - X^{n-1}/2
//       h^_k     = 2 Y_k^n - Y_k^{n-1}/2,      Y_k^{n+1} = d_k h^_k + d_k c_k P
//       G        = sum_k eta_k h^_k + (sum_k eta_k c_k) P          (compensated, FP64)
//       [(b0 + eta/De) I - eta (kappa~ . + . kappa~^T)] X^{n+1} = P - A(G) + zeta^{n+1} S
//       tau^{n+1} = (gamma/dt) (eta X^{n+1} - G)
//     The modes are streamed once: two levels read, one level written into the slot of
//     the older level.  The c x c local system (c = 3 or 6) is solved per lane by
//     Gaussian elimination with partial pivoting.
//   * SDIRK2 start-up (first step from rest of the modes): two stage solves with the
//     same local matrix; the level-0 and level-1 modes are written.
// The mode loop is a pure stream (no MFMA: about one flop per byte); global loads of
// the next mode are issued before the stores of the current one, so several KB per
// wave are in flight.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "tfs_internal.h"

namespace tfs {
namespace {

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
// Row exchanges are selects, so every lane runs the same instruction stream.
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
__device__ DiagAcc block_reduce(DiagAcc a) {
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

// One block folds the block partials in a fixed order.
__global__ __launch_bounds__(kBlock) void diag_finish_kernel(const double* __restrict__ part, int nparts,
                                                             double* __restrict__ diag) {
  DiagAcc a;
  for (int i = threadIdx.x; i < nparts; i += kBlock) {
    DiagAcc b;
    const double* q = part + (size_t)i * kNumDiag;
    b.mn1 = q[0]; b.mn2 = q[1]; b.mn3 = q[2]; b.mx = q[3]; b.sum = q[4]; b.cnt = q[5];
    diag_combine(a, b);
  }
  const DiagAcc r = block_reduce(a);
  if (threadIdx.x == 0) {
    diag[0] = r.mn1; diag[1] = r.mn2; diag[2] = r.mn3; diag[3] = r.mx; diag[4] = r.sum; diag[5] = r.cnt;
  }
}

// ------------------------------------------------------------------ BDF2 step
template <typename MT>
struct Bdf2Args {
  const double* ka;     // kappa_a [d*d][stride]
  const double* kb;     // kappa_b or null
  const double* Xn;     // X^n      [c][stride]
  double* Xm;           // X^{n-1} in, X^{n+1} out (same slot)
  const MT* Yn;         // Y^n slot (m * c * stride elements, tiled)
  MT* Ym;               // Y^{n-1} in, Y^{n+1} out (same slot)
  double* tau;          // [c][stride] or null
  const double* coef;   // [kNumCoef][m]
  double* part;         // block partials or null
  int64_t npts, stride, tile;
  int m;
  Bdf2Scalars s;
};

template <int D, typename MT, int V, bool FULL, bool DIAG>
__device__ __forceinline__ void bdf2_group(const Bdf2Args<MT>& a, int64_t p0, int nv, DiagAcc& acc) {
  constexpr int C = Sym<D>::C;
  const int64_t st = a.stride;
  const int m = a.m;

  // P = 2 X^n - X^{n-1}/2
  double P[C][V];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    double xn[V], xm[V];
    load_v<FULL, double, V>(a.Xn + s * st + p0, nv, xn);
    load_v<FULL, double, V>(a.Xm + s * st + p0, nv, xm);
#pragma unroll
    for (int v = 0; v < V; ++v) P[s][v] = 2.0 * xn[v] - 0.5 * xm[v];
  }

  // mode stream: the loads of mode k+1 are issued before the stores of mode k
  double Gs[C][V], Ge[C][V];
#pragma unroll
  for (int s = 0; s < C; ++s)
#pragma unroll
    for (int v = 0; v < V; ++v) { Gs[s][v] = 0.0; Ge[s][v] = 0.0; }

  // mode (k, s) of the group: tile base + (k C + s) T
  const int64_t T = a.tile;
  const int64_t toff = (p0 / T) * (int64_t)m * C * T + (p0 % T);
  const MT* yn0 = a.Yn + toff;
  MT* ym0 = a.Ym + toff;
  MT cn[C][V], cm[C][V];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    load_v<FULL, MT, V, true>(yn0 + s * T, nv, cn[s]);
    load_v<FULL, MT, V, true>(ym0 + s * T, nv, cm[s]);
  }
  for (int k = 0; k < m; ++k) {
    const double dk = a.coef[kRowD * m + k];
    const double dck = a.coef[kRowDC * m + k];
    const double ek = a.coef[kRowEta * m + k];
    MT nn[C][V], nm[C][V];
    if (k + 1 < m) {
      const MT* yn1 = yn0 + (int64_t)(k + 1) * C * T;
      const MT* ym1 = ym0 + (int64_t)(k + 1) * C * T;
#pragma unroll
      for (int s = 0; s < C; ++s) {
        load_v<FULL, MT, V, true>(yn1 + s * T, nv, nn[s]);
        load_v<FULL, MT, V, true>(ym1 + s * T, nv, nm[s]);
      }
    }
    MT* yo = ym0 + (int64_t)k * C * T;
#pragma unroll
    for (int s = 0; s < C; ++s) {
      MT out[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double h = 2.0 * (double)cn[s][v] - 0.5 * (double)cm[s][v];
        out[v] = (MT)(dk * h + dck * P[s][v]);
        two_sum_acc(Gs[s][v], Ge[s][v], mul_rn(ek, h));
      }
      store_v<FULL, MT, V, true>(yo + s * T, nv, out);
    }
    if (k + 1 < m) {
#pragma unroll
      for (int s = 0; s < C; ++s)
#pragma unroll
        for (int v = 0; v < V; ++v) { cn[s][v] = nn[s][v]; cm[s][v] = nm[s][v]; }
    }
  }

  // velocity gradient driving the step
  double kt[D * D][V];
#pragma unroll
  for (int q = 0; q < D * D; ++q) {
    double ka[V];
    load_v<FULL, double, V>(a.ka + q * st + p0, nv, ka);
    if (a.kb) {
      double kb[V];
      load_v<FULL, double, V>(a.kb + q * st + p0, nv, kb);
#pragma unroll
      for (int v = 0; v < V; ++v) kt[q][v] = 2.0 * ka[v] - kb[v];
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) kt[q][v] = ka[v];
    }
  }

  double Xout[C][V], Tout[C][V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    double k[D * D], G[C], AG[C], R[C];
#pragma unroll
    for (int q = 0; q < D * D; ++q) k[q] = kt[q][v];
#pragma unroll
    for (int s = 0; s < C; ++s) G[s] = (Gs[s][v] + Ge[s][v]) + a.s.s_ec * P[s][v];
    apply_K<D>(k, G, AG);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const int i = Sym<D>::i(s), j = Sym<D>::j(s);
      const double S = k[i * D + j] + k[j * D + i];
      R[s] = P[s][v] - (AG[s] - a.s.inv_De * G[s]) + a.s.zeta * S;
    }
    double M[C][C];
    build_M<D>(k, a.s.a_diag, a.s.eta, M);
    solve_pivot<C>(M, R);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      Xout[s][v] = R[s];
      Tout[s][v] = a.s.tau_scale * (a.s.eta * R[s] - G[s]);
    }
    if constexpr (DIAG) {
      if (FULL || v < nv) {
        double xs[C], ts[C];
#pragma unroll
        for (int s = 0; s < C; ++s) { xs[s] = Xout[s][v]; ts[s] = Tout[s][v]; }
        diag_point<D>(acc, xs, ts);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < C; ++s) {
    store_v<FULL, double, V>(a.Xm + s * st + p0, nv, Xout[s]);
    if (a.tau) store_v<FULL, double, V>(a.tau + s * st + p0, nv, Tout[s]);
  }
}

template <int D, typename MT, int V, bool DIAG>
__global__ __launch_bounds__(kBlock) void bdf2_kernel(const Bdf2Args<MT> a) {
  DiagAcc acc;
  const int64_t ngroups = (a.npts + V - 1) / V;
  const int64_t gstride = (int64_t)gridDim.x * kBlock;
  for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < ngroups; g += gstride) {
    const int64_t p0 = g * V;
    const int nv = (int)((a.npts - p0) < V ? (a.npts - p0) : V);
    if (nv == V) bdf2_group<D, MT, V, true, DIAG>(a, p0, nv, acc);
    else bdf2_group<D, MT, V, false, DIAG>(a, p0, nv, acc);
  }
  if constexpr (DIAG) {
    const DiagAcc r = block_reduce(acc);
    if (threadIdx.x == 0) write_partial(a.part, blockIdx.x, r);
  }
}

// ------------------------------------------------------------------ SDIRK2 start-up
template <typename MT>
struct StartArgs {
  const double* ka;  // kappa^0
  double* X;         // ring [2][c][stride]: reads slot 0, writes slot 1
  MT* Y;             // ring, 2 slots of m * c * stride elements (tiled): writes both slots
  double* tau;
  const double* coef;
  double* part;
  int64_t npts, stride, tile;
  int m;
  StartScalars s;
};

template <int D, typename MT, int V, bool FULL, bool DIAG>
__device__ __forceinline__ void start_group(const StartArgs<MT>& a, int64_t p0, int nv, DiagAcc& acc) {
  constexpr int C = Sym<D>::C;
  const int64_t st = a.stride;
  const int m = a.m;
  double X0[C][V], X1[C][V], X2[C][V];
#pragma unroll
  for (int s = 0; s < C; ++s) load_v<FULL, double, V>(a.X + s * st + p0, nv, X0[s]);
  double kt[D * D][V];
#pragma unroll
  for (int q = 0; q < D * D; ++q) load_v<FULL, double, V>(a.ka + q * st + p0, nv, kt[q]);

  double Tout[C][V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    double k[D * D], S[C], r[C], M[C][C], AX[C], x1[C];
#pragma unroll
    for (int q = 0; q < D * D; ++q) k[q] = kt[q][v];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const int i = Sym<D>::i(s), j = Sym<D>::j(s);
      S[s] = k[i * D + j] + k[j * D + i];
    }
    // stage 1: (I - h gs theta A) X1 = X0 + h gs theta S
#pragma unroll
    for (int s = 0; s < C; ++s) r[s] = X0[s][v] + a.s.src1 * S[s];
    build_M<D>(k, 1.0 + a.s.hgt * a.s.inv_De, a.s.hgt, M);
    solve_pivot<C>(M, r);
#pragma unroll
    for (int s = 0; s < C; ++s) { x1[s] = r[s]; X1[s][v] = r[s]; }
    // stage 2: (I - h gs theta A) X2 = X0 + sigma1 A(X1) + sigma2 S
    apply_K<D>(k, x1, AX);
#pragma unroll
    for (int s = 0; s < C; ++s)
      r[s] = X0[s][v] + a.s.sigma1 * (AX[s] - a.s.inv_De * x1[s]) + a.s.sigma2 * S[s];
    build_M<D>(k, 1.0 + a.s.hgt * a.s.inv_De, a.s.hgt, M);
    solve_pivot<C>(M, r);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      X2[s][v] = r[s];
      Tout[s][v] = a.s.gamma * (a.s.theta * r[s] - a.s.hr * x1[s]);
    }
    if constexpr (DIAG) {
      if (FULL || v < nv) {
        double xs[C], ts[C];
#pragma unroll
        for (int s = 0; s < C; ++s) { xs[s] = X2[s][v]; ts[s] = Tout[s][v]; }
        diag_point<D>(acc, xs, ts);
      }
    }
  }
#pragma unroll
  for (int s = 0; s < C; ++s) {
    store_v<FULL, double, V>(a.X + (C + s) * st + p0, nv, X2[s]);
    if (a.tau) store_v<FULL, double, V>(a.tau + s * st + p0, nv, Tout[s]);
  }
  // modes: Y_k^0 = -c_k X^0 (slot 0), Y_k^1 = u_k X^(1) + v_k X^(2) (slot 1)
  const int64_t T = a.tile;
  const int64_t toff = (p0 / T) * (int64_t)m * C * T + (p0 % T);
  MT* Y0 = a.Y + toff;
  MT* Y1 = a.Y + (int64_t)m * C * st + toff;
  for (int k = 0; k < m; ++k) {
    const double ck = a.coef[kRowC * m + k];
    const double uk = a.coef[kRowU * m + k];
    const double vk = a.coef[kRowV * m + k];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      MT o0[V], o1[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        o0[v] = (MT)(-ck * X0[s][v]);
        o1[v] = (MT)(uk * X1[s][v] + vk * X2[s][v]);
      }
      store_v<FULL, MT, V, true>(Y0 + ((int64_t)k * C + s) * T, nv, o0);
      store_v<FULL, MT, V, true>(Y1 + ((int64_t)k * C + s) * T, nv, o1);
    }
  }
}

template <int D, typename MT, int V, bool DIAG>
__global__ __launch_bounds__(kBlock) void start_kernel(const StartArgs<MT> a) {
  DiagAcc acc;
  const int64_t ngroups = (a.npts + V - 1) / V;
  const int64_t gstride = (int64_t)gridDim.x * kBlock;
  for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < ngroups; g += gstride) {
    const int64_t p0 = g * V;
    const int nv = (int)((a.npts - p0) < V ? (a.npts - p0) : V);
    if (nv == V) start_group<D, MT, V, true, DIAG>(a, p0, nv, acc);
    else start_group<D, MT, V, false, DIAG>(a, p0, nv, acc);
  }
  if constexpr (DIAG) {
    const DiagAcc r = block_reduce(acc);
    if (threadIdx.x == 0) write_partial(a.part, blockIdx.x, r);
  }
}

// ------------------------------------------------------------------ plain modes
template <typename MT>
__global__ __launch_bounds__(kBlock) void plain_kernel(const double* __restrict__ X, const MT* __restrict__ Y,
                                                       const double* __restrict__ coef, double* __restrict__ out,
                                                       int64_t npts, int64_t stride, int64_t tile, int m, int c) {
  const int64_t total = (int64_t)m * c * npts;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < total; t += (int64_t)gridDim.x * kBlock) {
    const int64_t p = t % npts;
    const int64_t ks = t / npts;
    const int s = (int)(ks % c);
    const int k = (int)(ks / c);
    const int64_t yi = ((p / tile) * m * c + ks) * tile + p % tile;
    out[ks * stride + p] = (double)Y[yi] + coef[kRowC * m + k] * X[s * stride + p];
  }
}

// ------------------------------------------------------------------ launch helpers
int grid_for(const tfs_plan_s* p, int64_t ngroups) {
  const int64_t cap = (int64_t)p->num_cus * p->grid_per_cu;
  int64_t g = (ngroups + kBlock - 1) / kBlock;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

bool aligned(const void* ptr, size_t bytes) { return ptr == nullptr || ((uintptr_t)ptr % bytes) == 0; }

// Points per lane: the requested width, else the widest one (4 for FP32 modes, 2 for
// FP64: 16-byte mode accesses, fastest on MI355X) for which every plane start and every
// group start is aligned to the vector size of each field (modes: V * sizeof(MT); FP64
// fields: V * 8).
template <int D, typename MT>
int pick_vec(const tfs_plan_s* p, const void* k0, const void* k1, const void* X, const void* Y,
             const void* tau) {
  const int widest = sizeof(MT) == 4 ? 4 : 2;
  const int cand[3] = {widest, 2, 1};
  for (int V : cand) {
    if (V > widest) continue;
    if (p->vec_override && V != p->vec_override) continue;
    if (p->stride % V || p->tile % V) continue;
    const size_t bm = (size_t)V * sizeof(MT), bd = (size_t)V * 8;
    if (aligned(k0, bd) && aligned(k1, bd) && aligned(X, bd) && aligned(Y, bm) && aligned(tau, bd)) return V;
  }
  return 1;
}

template <int D, typename MT, int V>
hipError_t bdf2_go(const tfs_plan_s* p, const Bdf2Args<MT>& a, bool diag, double* diag_out) {
  const int64_t ngroups = (a.npts + V - 1) / V;
  const int grid = grid_for(p, ngroups);
  if (diag) {
    hipLaunchKernelGGL((bdf2_kernel<D, MT, V, true>), dim3(grid), dim3(kBlock), 0, p->stream, a);
    hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(kBlock), 0, p->stream, a.part, grid, diag_out);
  } else {
    hipLaunchKernelGGL((bdf2_kernel<D, MT, V, false>), dim3(grid), dim3(kBlock), 0, p->stream, a);
  }
  return hipGetLastError();
}

template <int D, typename MT>
hipError_t bdf2_dispatch(const tfs_plan_s* p, int64_t n, const double* ka, const double* kb, double* X, void* Y,
                         double* tau, double* diag) {
  constexpr int C = Sym<D>::C;
  const int64_t st = p->stride;
  const int sn = (int)(n % 2), sm = 1 - sn;
  Bdf2Args<MT> a;
  a.ka = ka;
  a.kb = kb;
  a.Xn = X + (int64_t)sn * C * st;
  a.Xm = X + (int64_t)sm * C * st;
  MT* Yb = static_cast<MT*>(Y);
  a.Yn = Yb + (int64_t)sn * p->m * C * st;
  a.Ym = Yb + (int64_t)sm * p->m * C * st;
  a.tau = tau;
  a.coef = p->d_coef;
  a.part = p->d_part;
  a.npts = p->npoints;
  a.stride = st;
  a.tile = p->tile;
  a.m = p->m;
  a.s.a_diag = p->a_diag;
  a.s.eta = p->eta;
  a.s.s_ec = p->s_ec;
  a.s.inv_De = 1.0 / p->De;
  a.s.zeta = p->zeta[n + 1];
  a.s.tau_scale = p->tau_scale;
  const int V = pick_vec<D, MT>(p, ka, kb, X, Y, tau);
  const bool dg = diag != nullptr;
  if constexpr (sizeof(MT) == 4) {
    if (V == 4) return bdf2_go<D, MT, 4>(p, a, dg, diag);
  }
  if (V == 2) return bdf2_go<D, MT, 2>(p, a, dg, diag);
  return bdf2_go<D, MT, 1>(p, a, dg, diag);
}

template <int D, typename MT, int V>
hipError_t start_go(const tfs_plan_s* p, const StartArgs<MT>& a, bool diag, double* diag_out) {
  const int64_t ngroups = (a.npts + V - 1) / V;
  const int grid = grid_for(p, ngroups);
  if (diag) {
    hipLaunchKernelGGL((start_kernel<D, MT, V, true>), dim3(grid), dim3(kBlock), 0, p->stream, a);
    hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(kBlock), 0, p->stream, a.part, grid, diag_out);
  } else {
    hipLaunchKernelGGL((start_kernel<D, MT, V, false>), dim3(grid), dim3(kBlock), 0, p->stream, a);
  }
  return hipGetLastError();
}

template <int D, typename MT>
hipError_t start_dispatch(const tfs_plan_s* p, const double* ka, double* X, void* Y, double* tau, double* diag) {
  StartArgs<MT> a;
  a.ka = ka;
  a.X = X;
  a.Y = static_cast<MT*>(Y);
  a.tau = tau;
  a.coef = p->d_coef;
  a.part = p->d_part;
  a.npts = p->npoints;
  a.stride = p->stride;
  a.tile = p->tile;
  a.m = p->m;
  a.s.hgt = p->hg * p->theta;
  a.s.inv_De = 1.0 / p->De;
  a.s.src1 = p->hg * p->theta;
  a.s.sigma1 = p->sigma1;
  a.s.sigma2 = p->sigma2;
  a.s.gamma = p->gamma;
  a.s.theta = p->theta;
  a.s.hr = p->hr;
  const int V = pick_vec<D, MT>(p, ka, nullptr, X, Y, tau);
  const bool dg = diag != nullptr;
  if constexpr (sizeof(MT) == 4) {
    if (V == 4) return start_go<D, MT, 4>(p, a, dg, diag);
  }
  if (V == 2) return start_go<D, MT, 2>(p, a, dg, diag);
  return start_go<D, MT, 1>(p, a, dg, diag);
}

}  // namespace

int max_blocks(const tfs_plan_s* p) { return p->num_cus * kMaxBlocksPerCU; }

hipError_t launch_bdf2(const tfs_plan_s* p, int64_t n, const double* ka, const double* kb, double* X, void* Y,
                       double* tau, double* diag) {
  if (p->npoints == 0) {
    if (diag) hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(kBlock), 0, p->stream, p->d_part, 0, diag);
    return hipGetLastError();
  }
  if (p->precision == TFS_FP64)
    return p->d == 2 ? bdf2_dispatch<2, double>(p, n, ka, kb, X, Y, tau, diag)
                     : bdf2_dispatch<3, double>(p, n, ka, kb, X, Y, tau, diag);
  return p->d == 2 ? bdf2_dispatch<2, float>(p, n, ka, kb, X, Y, tau, diag)
                   : bdf2_dispatch<3, float>(p, n, ka, kb, X, Y, tau, diag);
}

hipError_t launch_startup(const tfs_plan_s* p, const double* ka, double* X, void* Y, double* tau, double* diag) {
  if (p->npoints == 0) {
    if (diag) hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(kBlock), 0, p->stream, p->d_part, 0, diag);
    return hipGetLastError();
  }
  if (p->precision == TFS_FP64)
    return p->d == 2 ? start_dispatch<2, double>(p, ka, X, Y, tau, diag)
                     : start_dispatch<3, double>(p, ka, X, Y, tau, diag);
  return p->d == 2 ? start_dispatch<2, float>(p, ka, X, Y, tau, diag)
                   : start_dispatch<3, float>(p, ka, X, Y, tau, diag);
}

hipError_t launch_modes_to_plain(const tfs_plan_s* p, int slot, const double* X, const void* Y, double* Xk) {
  if (p->npoints == 0) return hipSuccess;
  const int64_t st = p->stride;
  const double* Xs = X + (int64_t)slot * p->c * st;
  const int64_t total = (int64_t)p->m * p->c * p->npoints;
  int grid = (int)((total + kBlock - 1) / kBlock);
  if (grid > 65536) grid = 65536;
  if (p->precision == TFS_FP64) {
    const double* Ys = static_cast<const double*>(Y) + (int64_t)slot * p->m * p->c * st;
    hipLaunchKernelGGL(plain_kernel<double>, dim3(grid), dim3(kBlock), 0, p->stream, Xs, Ys, p->d_coef, Xk,
                       p->npoints, st, p->tile, p->m, p->c);
  } else {
    const float* Ys = static_cast<const float*>(Y) + (int64_t)slot * p->m * p->c * st;
    hipLaunchKernelGGL(plain_kernel<float>, dim3(grid), dim3(kBlock), 0, p->stream, Xs, Ys, p->d_coef, Xk,
                       p->npoints, st, p->tile, p->m, p->c);
  }
  return hipGetLastError();
}

}  // namespace tfs

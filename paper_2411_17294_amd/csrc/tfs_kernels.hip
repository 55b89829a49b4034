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
//   * Exponential-mode step (an extension, not the paper's scheme): every mode solved
//     exactly for X linear on the step, one mode level updated in place, and the state
//     integrated as X^{n+1} - X^n = A(sum_k (X_k^{n+1} - X_k^n)) + zeta S.
// The mode loop is a pure stream (no MFMA: about one flop per byte); global loads of
// the next mode are issued before the stores of the current one, so several KB per
// wave are in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

#include "tfs_device.h"
#include "tfs_internal.h"

namespace tfs {
namespace {
using namespace dev;

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
// Spatial form (eps Laplace where it is diagonal): each point is one coefficient of a
// field in a basis of Laplace eigenfunctions.  -eps Laplace acts on it as the extra
// relaxation rate eps |xi|^2, and only the constant function's coefficient carries the
// mass-mode source (the mass mode is the constant 1).
struct SpatialArgs {
  const double* rate;   // [stride] extra relaxation rate per point, or null (none)
  int64_t src;          // the point with the mass-mode source, or -1 (every point)
};

// The extra rate and the source weight (1 or 0) of the lane's V points.
template <int V>
__device__ __forceinline__ void load_spatial(const SpatialArgs& sp, const WaveAddr& w, double (&rate)[V],
                                             double (&srcw)[V]) {
  if (sp.rate) {
    load_v<true, double, V>(at(sp.rate + w.pw, w.ox), V, rate);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) rate[v] = 0.0;
  }
  const int64_t p0 = w.pw + (int64_t)(w.ox / 8);
#pragma unroll
  for (int v = 0; v < V; ++v) srcw[v] = (sp.src < 0 || p0 + v == sp.src) ? 1.0 : 0.0;
}

template <typename MT, typename KT>
struct Bdf2Args {
  const KT* ka;         // kappa_a [d*d][stride] (FP64, or FP32 for an FP32-kappa plan)
  const KT* kb;         // kappa_b or null
  const double* Xn;     // X^n      [c][stride]
  const double* Xm;     // X^{n-1}  [c][stride]
  const double* Xmm;    // X^{n-2}  [c][stride] (shifted mode form; null: zero)
  double* Xo;           // X^{n+1}  [c][stride] (may be Xm or Xmm: each lane reads before it writes)
  const MT* Yn;         // Y^n      (m * c * stride elements, tiled; Z^n in the shifted form)
  const MT* Ym;         // Y^{n-1}
  MT* Yo;               // Y^{n+1}  (may be Ym, same rule)
  double* tau;          // [c][stride] or null
  const double* coef;   // [kNumCoef][m]
  double* part;         // block partials or null (this launch writes part[part0 + block])
  int64_t p_begin;      // first point of this launch
  int64_t ngroups;      // groups of V points from p_begin
  int64_t stride, tile;
  int m, part0;
  Bdf2Scalars s;
  SpatialArgs sp;
};

// SPLIT: the step without its local solve, for a caller that solves a spatially coupled
// system for X^{n+1}: the modes advance as usual (in the Y-form they do not depend on
// X^{n+1}), the point's right-hand side R goes to Xo and the history combination G to tau.
// ZF: the shifted mode form Z_k^j = Y_k^j - beta_k X^{j-1}: the history is read back as
// h^_k = 2 Z_k^n - Z_k^{n-1}/2 + beta_k B with B = 2 X^{n-1} - X^{n-2}/2, and the new level is
// stored as Z_k^{n+1} = d_k h^_k + d_k c_k P - beta_k X^n (still independent of X^{n+1}).
template <int D, typename MT, typename KT, int V, bool DIAG, bool SP, bool SPLIT = false, bool ZF = false>
__device__ __forceinline__ void bdf2_group(const Bdf2Args<MT, KT>& a, const WaveAddr& w, DiagAcc& acc) {
  constexpr int C = Sym<D>::C;
  constexpr int CZ = ZF ? C : 1;
  const int64_t st = a.stride;
  const int m = a.m;
  const int64_t T = a.tile;

  // P = 2 X^n - X^{n-1}/2 (and B = 2 X^{n-1} - X^{n-2}/2 and X^n in the shifted form)
  double P[C][V], B[CZ][V], Xc[CZ][V];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    double xn[V], xm[V];
    load_v<true, double, V>(at(a.Xn + s * st + w.pw, w.ox), V, xn);
    load_v<true, double, V>(at(a.Xm + s * st + w.pw, w.ox), V, xm);
#pragma unroll
    for (int v = 0; v < V; ++v) P[s][v] = 2.0 * xn[v] - 0.5 * xm[v];
    if constexpr (ZF) {
      double xmm[V];
      if (a.Xmm) {
        load_v<true, double, V>(at(a.Xmm + s * st + w.pw, w.ox), V, xmm);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) xmm[v] = 0.0;
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        B[s][v] = 2.0 * xm[v] - 0.5 * xmm[v];
        Xc[s][v] = xn[v];
      }
    }
  }

  // mode stream: the loads of mode k+1 are issued before the stores of mode k
  double Gs[C][V], Ge[C][V];
#pragma unroll
  for (int s = 0; s < C; ++s)
#pragma unroll
    for (int v = 0; v < V; ++v) { Gs[s][v] = 0.0; Ge[s][v] = 0.0; }

  const MT* yn0 = a.Yn + w.tw;
  const MT* ym0 = a.Ym + w.tw;
  MT* yo0 = a.Yo + w.tw;
  MT cn[C][V], cm[C][V];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    load_v<true, MT, V, true>(at(yn0 + s * T, w.om), V, cn[s]);
    load_v<true, MT, V, true>(at(ym0 + s * T, w.om), V, cm[s]);
  }
  for (int k = 0; k < m; ++k) {
    const double dk = load_uniform(a.coef + kRowD * m + k);
    const double dck = load_uniform(a.coef + kRowDC * m + k);
    const double ek = load_uniform(a.coef + kRowEta * m + k);
    const double bk = ZF ? load_uniform(a.coef + kRowBeta * m + k) : 0.0;
    MT nn[C][V], nm[C][V];
    if (k + 1 < m) {
      const int64_t o = (int64_t)(k + 1) * C * T;
      const uint32_t om = opaque(w.om);
#pragma unroll
      for (int s = 0; s < C; ++s) {
        load_v<true, MT, V, true>(at(yn0 + o + s * T, om), V, nn[s]);
        load_v<true, MT, V, true>(at(ym0 + o + s * T, om), V, nm[s]);
      }
    }
    MT* yo = yo0 + (int64_t)k * C * T;
    const uint32_t om = opaque(w.om);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      MT out[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        double h = 2.0 * (double)cn[s][v] - 0.5 * (double)cm[s][v];
        if constexpr (ZF) {
          h += bk * B[s][v];
          out[v] = (MT)(dk * h + (dck * P[s][v] - bk * Xc[s][v]));
        } else {
          out[v] = (MT)(dk * h + dck * P[s][v]);
        }
        two_sum_acc(Gs[s][v], Ge[s][v], mul_rn(ek, h));
      }
      store_v<true, MT, V, true>(at(yo + s * T, om), V, out);
    }
    if (k + 1 < m) {
#pragma unroll
      for (int s = 0; s < C; ++s)
#pragma unroll
        for (int v = 0; v < V; ++v) { cn[s][v] = nn[s][v]; cm[s][v] = nm[s][v]; }
    }
  }

  // velocity gradient driving the step (read in its storage precision, extrapolated in FP64)
  double kt[D * D][V];
  const uint32_t kx = field_off<KT>(w.ox);
#pragma unroll
  for (int q = 0; q < D * D; ++q) {
    KT ka[V];
    load_v<true, KT, V>(at(a.ka + q * st + w.pw, kx), V, ka);
    if (a.kb) {
      KT kb[V];
      load_v<true, KT, V>(at(a.kb + q * st + w.pw, kx), V, kb);
#pragma unroll
      for (int v = 0; v < V; ++v) kt[q][v] = 2.0 * (double)ka[v] - (double)kb[v];
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) kt[q][v] = (double)ka[v];
    }
  }

  double rate[V], srcw[V];
  if constexpr (SP) load_spatial<V>(a.sp, w, rate, srcw);
  double Xout[C][V], Tout[C][V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    double k[D * D], G[C], AG[C], R[C];
    // relaxation plus the spatial rate; the mass-mode source; the diagonal of M
    const double idv = SP ? a.s.inv_De + rate[v] : a.s.inv_De;
    const double zw = SP ? a.s.zeta * srcw[v] : a.s.zeta;
    const double ad = SP ? a.s.a_diag + a.s.eta * rate[v] : a.s.a_diag;
#pragma unroll
    for (int q = 0; q < D * D; ++q) k[q] = kt[q][v];
#pragma unroll
    for (int s = 0; s < C; ++s) G[s] = (Gs[s][v] + Ge[s][v]) + a.s.s_ec * P[s][v];
    apply_K<D>(k, G, AG);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const int i = Sym<D>::i(s), j = Sym<D>::j(s);
      const double S = k[i * D + j] + k[j * D + i];
      R[s] = P[s][v] - (AG[s] - idv * G[s]) + zw * S;
    }
    if constexpr (SPLIT) {
#pragma unroll
      for (int s = 0; s < C; ++s) {
        Xout[s][v] = R[s];
        Tout[s][v] = G[s];
      }
      continue;
    }
    double M[C][C];
    build_M<D>(k, ad, a.s.eta, M);
    solve_pivot<C>(M, R);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      Xout[s][v] = R[s];
      Tout[s][v] = a.s.tau_scale * (a.s.eta * R[s] - G[s]);
    }
    if constexpr (DIAG) {
      double xs[C], ts[C];
#pragma unroll
      for (int s = 0; s < C; ++s) { xs[s] = Xout[s][v]; ts[s] = Tout[s][v]; }
      diag_point<D>(acc, xs, ts);
    }
  }
#pragma unroll
  for (int s = 0; s < C; ++s) {
    store_v<true, double, V>(at(a.Xo + s * st + w.pw, w.ox), V, Xout[s]);
    if (a.tau) store_v<true, double, V>(at(a.tau + s * st + w.pw, w.ox), V, Tout[s]);
  }
}

// Groups [0, ngroups) of V points from p_begin, 64 consecutive groups per wave; the
// caller launches a V = 1 pass for the points after the last whole group.
template <int D, typename MT, typename KT, int V, bool DIAG, bool SP, bool SPLIT = false, bool ZF = false>
__global__ __launch_bounds__(kBlock) void bdf2_kernel(const Bdf2Args<MT, KT> a) {
  constexpr int C = Sym<D>::C;
  DiagAcc acc;
  const int lane = threadIdx.x % 64;
  const int64_t nwaves = (a.ngroups + 63) / 64;
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / 64);
  for (int64_t wv = wave_uniform((int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64); wv < nwaves;
       wv += wstride) {
    if (wv * 64 + lane < a.ngroups)
      bdf2_group<D, MT, KT, V, DIAG, SP, SPLIT, ZF>(a, wave_addr<MT, C, V>(a.p_begin + wv * 64 * V, lane, a.tile, a.m),
                                                    acc);
  }
  if constexpr (DIAG) {
    const DiagAcc r = block_reduce(acc);
    if (threadIdx.x == 0) write_partial(a.part, a.part0 + blockIdx.x, r);
  }
}

// ------------------------------------------------------------------ SDIRK2 start-up
template <typename MT, typename KT>
struct StartArgs {
  const KT* ka;      // kappa^0
  const double* X0;  // X^0 [c][stride]
  double* X1;        // X^1 [c][stride] (out)
  MT* Y0;            // Y^0 (m * c * stride elements, tiled; out)
  MT* Y1;            // Y^1 (out)
  double* tau;
  const double* coef;
  double* part;
  int64_t p_begin, ngroups;
  int64_t stride, tile;
  int m, part0;
  int zform;         // shifted mode form: Z^1 = Y^1 - beta_k X^0 (Z^0 = Y^0: X^{-1} = 0)
  StartScalars s;
  SpatialArgs sp;
};

template <int D, typename MT, typename KT, int V, bool DIAG, bool SP>
__device__ __forceinline__ void start_group(const StartArgs<MT, KT>& a, const WaveAddr& w, DiagAcc& acc) {
  constexpr int C = Sym<D>::C;
  const int64_t st = a.stride;
  const int m = a.m;
  double X0[C][V], X1[C][V], X2[C][V];
#pragma unroll
  for (int s = 0; s < C; ++s) load_v<true, double, V>(at(a.X0 + s * st + w.pw, w.ox), V, X0[s]);
  double kt[D * D][V];
#pragma unroll
  for (int q = 0; q < D * D; ++q) {
    KT x[V];
    load_v<true, KT, V>(at(a.ka + q * st + w.pw, field_off<KT>(w.ox)), V, x);
#pragma unroll
    for (int v = 0; v < V; ++v) kt[q][v] = (double)x[v];
  }

  double rate[V], srcw[V];
  if constexpr (SP) load_spatial<V>(a.sp, w, rate, srcw);
  double Tout[C][V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    double k[D * D], S[C], r[C], M[C][C], AX[C], x1[C];
    // relaxation plus the spatial rate; the mass-mode source of the two stages
    const double idv = SP ? a.s.inv_De + rate[v] : a.s.inv_De;
    const double s1 = SP ? a.s.src1 * srcw[v] : a.s.src1;
    const double s2 = SP ? a.s.sigma2 * srcw[v] : a.s.sigma2;
#pragma unroll
    for (int q = 0; q < D * D; ++q) k[q] = kt[q][v];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const int i = Sym<D>::i(s), j = Sym<D>::j(s);
      S[s] = k[i * D + j] + k[j * D + i];
    }
    // stage 1: (I - h gs theta A) X1 = X0 + h gs theta S
#pragma unroll
    for (int s = 0; s < C; ++s) r[s] = X0[s][v] + s1 * S[s];
    build_M<D>(k, 1.0 + a.s.hgt * idv, a.s.hgt, M);
    solve_pivot<C>(M, r);
#pragma unroll
    for (int s = 0; s < C; ++s) { x1[s] = r[s]; X1[s][v] = r[s]; }
    // stage 2: (I - h gs theta A) X2 = X0 + sigma1 A(X1) + sigma2 S
    apply_K<D>(k, x1, AX);
#pragma unroll
    for (int s = 0; s < C; ++s)
      r[s] = X0[s][v] + a.s.sigma1 * (AX[s] - idv * x1[s]) + s2 * S[s];
    build_M<D>(k, 1.0 + a.s.hgt * idv, a.s.hgt, M);
    solve_pivot<C>(M, r);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      X2[s][v] = r[s];
      Tout[s][v] = a.s.gamma * (a.s.theta * r[s] - a.s.hr * x1[s]);
    }
    if constexpr (DIAG) {
      double xs[C], ts[C];
#pragma unroll
      for (int s = 0; s < C; ++s) { xs[s] = X2[s][v]; ts[s] = Tout[s][v]; }
      diag_point<D>(acc, xs, ts);
    }
  }
#pragma unroll
  for (int s = 0; s < C; ++s) {
    store_v<true, double, V>(at(a.X1 + s * st + w.pw, w.ox), V, X2[s]);
    if (a.tau) store_v<true, double, V>(at(a.tau + s * st + w.pw, w.ox), V, Tout[s]);
  }
  // modes: Y_k^0 = -c_k X^0 (slot 0), Y_k^1 = u_k X^(1) + v_k X^(2) (slot 1); in the
  // shifted form level 1 is stored less beta_k X^0
  const int64_t T = a.tile;
  MT* Y0 = a.Y0 + w.tw;
  MT* Y1 = a.Y1 + w.tw;
  for (int k = 0; k < m; ++k) {
    const double ck = load_uniform(a.coef + kRowC * m + k);
    const double uk = load_uniform(a.coef + kRowU * m + k);
    const double vk = load_uniform(a.coef + kRowV * m + k);
    const double bk = a.zform ? load_uniform(a.coef + kRowBeta * m + k) : 0.0;
#pragma unroll
    for (int s = 0; s < C; ++s) {
      MT o0[V], o1[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        o0[v] = (MT)(-ck * X0[s][v]);
        o1[v] = (MT)((uk * X1[s][v] + vk * X2[s][v]) - bk * X0[s][v]);
      }
      store_v<true, MT, V, true>(at(Y0 + ((int64_t)k * C + s) * T, w.om), V, o0);
      store_v<true, MT, V, true>(at(Y1 + ((int64_t)k * C + s) * T, w.om), V, o1);
    }
  }
}

template <int D, typename MT, typename KT, int V, bool DIAG, bool SP>
__global__ __launch_bounds__(kBlock) void start_kernel(const StartArgs<MT, KT> a) {
  constexpr int C = Sym<D>::C;
  DiagAcc acc;
  const int lane = threadIdx.x % 64;
  const int64_t nwaves = (a.ngroups + 63) / 64;
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / 64);
  for (int64_t wv = wave_uniform((int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64); wv < nwaves;
       wv += wstride) {
    if (wv * 64 + lane < a.ngroups)
      start_group<D, MT, KT, V, DIAG, SP>(a, wave_addr<MT, C, V>(a.p_begin + wv * 64 * V, lane, a.tile, a.m), acc);
  }
  if constexpr (DIAG) {
    const DiagAcc r = block_reduce(acc);
    if (threadIdx.x == 0) write_partial(a.part, a.part0 + blockIdx.x, r);
  }
}

// ------------------------------------------------------------------ exponential-mode step
// Each mode is advanced exactly for X linear on the step (TFS_SCHEME_EXP):
//   Y_k^{n+1} = e_k Y_k^n + f_k X^n                      (Y_k = X_k - q_k X, stored in place)
//   H  = sum_k (1 - e_k) Y_k^n + s_h X^n                  (X^{n+1} - X^n = A(q X^{n+1} - H) + zeta S)
//   G  = sum_k lambda_k dt Y_k^{n+1}                      (dt D^{1-alpha} X^{n+1} = eta_e X^{n+1} - G)
//   [(1 + q/De) I - q (kappa~ . + . kappa~^T)] X^{n+1} = X^n - A(H) + zeta S
//   tau^{n+1} = (gamma/dt)(eta_e X^{n+1} - G)
// H and G are compensated FP64 sums; one read and one write per mode-component.
// Mode loads issued ahead of the arithmetic in the exponential-mode step.
constexpr int kExpAhead = 2;

template <typename MT, typename KT>
struct ExpArgs {
  const KT* ka;         // kappa_a [d*d][stride]
  const KT* kb;         // kappa_b or null
  const double* Xn;     // X^n     [c][stride]
  double* Xo;           // X^{n+1} [c][stride]
  const MT* Yn;         // Y^n (m * c * stride elements, tiled); not read at n = 0
  MT* Yo;               // Y^{n+1} (may be Yn: each lane reads a mode before writing it)
  double* tau;          // [c][stride] or null
  double* Hout;         // SPLIT: H [c][stride]
  const double* coef;   // [kNumCoef][m], ExpRow order
  double* part;         // block partials or null (this launch writes part[part0 + block])
  int64_t p_begin, ngroups;
  int64_t stride, tile;
  int m, part0;
  ExpScalars s;
  SpatialArgs sp;
};

// SPLIT: the step without its local solve, for a caller that solves a spatially coupled
// system: X^{n+1} receives each point's right-hand side R, tau the compensated G and Hout the
// H of the local system (the modes are written as usual: they do not depend on X^{n+1}).
template <int D, typename MT, typename KT, int V, bool DIAG, bool SP, bool SPLIT = false>
__device__ __forceinline__ void exp_group(const ExpArgs<MT, KT>& a, const WaveAddr& w, DiagAcc& acc) {
  constexpr int C = Sym<D>::C;
  const int64_t st = a.stride;
  const int m = a.m;
  const int64_t T = a.tile;
  const bool first = a.s.first != 0;

  double Xc[C][V];
#pragma unroll
  for (int s = 0; s < C; ++s) load_v<true, double, V>(at(a.Xn + s * st + w.pw, w.ox), V, Xc[s]);

  // H enters the solve only (plain FP64 sum); G is the stress's near-cancelling term
  // (compensated)
  double H[C][V], Gs[C][V], Ge[C][V];
#pragma unroll
  for (int s = 0; s < C; ++s)
#pragma unroll
    for (int v = 0; v < V; ++v) { H[s][v] = 0.0; Gs[s][v] = 0.0; Ge[s][v] = 0.0; }

  // one read stream: the loads run kExpAhead modes ahead of the arithmetic
  const MT* yn0 = a.Yn + w.tw;
  MT* yo0 = a.Yo + w.tw;
  MT buf[kExpAhead + 1][C][V];
  if (!first) {
#pragma unroll
    for (int j = 0; j < kExpAhead; ++j) {
      if (j < m) {
        const uint32_t om = opaque(w.om);
        const MT* b = opaque_ptr(yn0 + (int64_t)j * C * T);
#pragma unroll
        for (int s = 0; s < C; ++s) load_v<true, MT, V, true>(at(b + s * T, om), V, buf[j][s]);
      }
    }
  }
  for (int k = 0; k < m; ++k) {
    const double ek = load_uniform(a.coef + kRowE * m + k);
    const double fk = load_uniform(a.coef + kRowF * m + k);
    const double lk = load_uniform(a.coef + kRowLdt * m + k);
    const double qk = load_uniform(a.coef + kRowQ * m + k);
    const double ok = load_uniform(a.coef + kRowOneME * m + k);
    if (!first && k + kExpAhead < m) {
      const uint32_t om = opaque(w.om);
      const MT* b = opaque_ptr(yn0 + (int64_t)(k + kExpAhead) * C * T);
#pragma unroll
      for (int s = 0; s < C; ++s) load_v<true, MT, V, true>(at(b + s * T, om), V, buf[kExpAhead][s]);
    }
    const uint32_t om = opaque(w.om);
    MT* bo = opaque_ptr(yo0 + (int64_t)k * C * T);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      MT out[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double y = first ? -qk * Xc[s][v] : (double)buf[0][s][v];
        out[v] = (MT)(ek * y + fk * Xc[s][v]);
        H[s][v] += ok * y;
        two_sum_acc(Gs[s][v], Ge[s][v], mul_rn(lk, (double)out[v]));
      }
      store_v<true, MT, V, true>(at(bo + s * T, om), V, out);
    }
    if (!first) {
#pragma unroll
      for (int j = 0; j < kExpAhead; ++j)
#pragma unroll
        for (int s = 0; s < C; ++s)
#pragma unroll
          for (int v = 0; v < V; ++v) buf[j][s][v] = buf[j + 1][s][v];
    }
  }

  // the local solve point by point (kappa loaded per point): one c x c system live at a time.
  // X^{n+1} and tau are stored V-wide at the end; in 3-D the finished points wait in LDS
  // instead of registers.
  constexpr bool kLds = (D == 3) && !SPLIT;
  __shared__ double stage[(kLds && V > 1) ? 2 * C * (V - 1) : 1][kBlock];
  double Xout[C][V], Tout[C][V], Hsp[SPLIT ? C : 1][V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint32_t ox = w.ox + v * 8;
    double k[D * D], Hv[C], AH[C], R[C];
#pragma unroll
    for (int q = 0; q < D * D; ++q) {
      KT x[1];
      load_v<true, KT, 1>(at(a.ka + q * st + w.pw, field_off<KT>(ox)), 1, x);
      k[q] = (double)x[0];
      if (a.kb) {
        load_v<true, KT, 1>(at(a.kb + q * st + w.pw, field_off<KT>(ox)), 1, x);
        k[q] = a.s.fa * k[q] + a.s.fb * (double)x[0];
      }
    }
    double rate = 0.0, srcw = 1.0;                 // spatial form: extra rate, source weight
    if constexpr (SP) {
      if (a.sp.rate) {
        double x[1];
        load_v<true, double, 1>(at(a.sp.rate + w.pw, ox), 1, x);
        rate = x[0];
      }
      srcw = (a.sp.src < 0 || w.pw + (int64_t)(ox / 8) == a.sp.src) ? 1.0 : 0.0;
    }
    const double idv = SP ? a.s.inv_De + rate : a.s.inv_De;
    const double zw = SP ? a.s.zeta * srcw : a.s.zeta;
    const double ad = SP ? a.s.a_diag + a.s.q * rate : a.s.a_diag;
#pragma unroll
    for (int s = 0; s < C; ++s) Hv[s] = H[s][v] + a.s.s_h * Xc[s][v];
    apply_K<D>(k, Hv, AH);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const int i = Sym<D>::i(s), j = Sym<D>::j(s);
      const double S = k[i * D + j] + k[j * D + i];
      R[s] = Xc[s][v] - (AH[s] - idv * Hv[s]) + zw * S;
    }
    if constexpr (SPLIT) {
#pragma unroll
      for (int s = 0; s < C; ++s) {
        Xout[s][v] = R[s];
        Tout[s][v] = Gs[s][v] + Ge[s][v];
        Hsp[s][v] = Hv[s];
      }
      continue;
    }
    double M[C][C];
    build_M<D>(k, ad, a.s.q, M);
    solve_pivot<C>(M, R);
    double ts[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      ts[s] = a.s.tau_scale * (a.s.eta_e * R[s] - (Gs[s][v] + Ge[s][v]));
      if (kLds && v + 1 < V) {
        stage[(2 * s) * (V - 1) + v][threadIdx.x] = R[s];
        stage[(2 * s + 1) * (V - 1) + v][threadIdx.x] = ts[s];
      } else {
        Xout[s][v] = R[s];
        Tout[s][v] = ts[s];
      }
    }
    if constexpr (DIAG) diag_point<D>(acc, R, ts);
  }
#pragma unroll
  for (int s = 0; s < C; ++s) {
    if constexpr (kLds) {
#pragma unroll
      for (int v = 0; v + 1 < V; ++v) {
        Xout[s][v] = stage[(2 * s) * (V - 1) + v][threadIdx.x];
        Tout[s][v] = stage[(2 * s + 1) * (V - 1) + v][threadIdx.x];
      }
    }
    store_v<true, double, V>(at(a.Xo + s * st + w.pw, w.ox), V, Xout[s]);
    if (a.tau) store_v<true, double, V>(at(a.tau + s * st + w.pw, w.ox), V, Tout[s]);
    if constexpr (SPLIT) store_v<true, double, V>(at(a.Hout + s * st + w.pw, w.ox), V, Hsp[s]);
  }
}

template <int D, typename MT, typename KT, int V, bool DIAG, bool SP, bool SPLIT = false>
__global__ __launch_bounds__(kBlock) void exp_kernel(const ExpArgs<MT, KT> a) {
  constexpr int C = Sym<D>::C;
  DiagAcc acc;
  const int lane = threadIdx.x % 64;
  const int64_t nwaves = (a.ngroups + 63) / 64;
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / 64);
  for (int64_t wv = wave_uniform((int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64); wv < nwaves;
       wv += wstride) {
    if (wv * 64 + lane < a.ngroups)
      exp_group<D, MT, KT, V, DIAG, SP, SPLIT>(a, wave_addr<MT, C, V>(a.p_begin + wv * 64 * V, lane, a.tile, a.m),
                                               acc);
  }
  if constexpr (DIAG) {
    const DiagAcc r = block_reduce(acc);
    if (threadIdx.x == 0) write_partial(a.part, a.part0 + blockIdx.x, r);
  }
}

// ------------------------------------------------------------------ plain modes
// X_k = Y_k + c_k X^j (+ beta_k X^{j-1} in the shifted form, Xm null: zero).
template <typename MT>
__global__ __launch_bounds__(kBlock) void plain_kernel(const double* __restrict__ X, const double* __restrict__ Xm,
                                                       const MT* __restrict__ Y, const double* __restrict__ coef,
                                                       double* __restrict__ out, int64_t npts, int64_t stride,
                                                       int64_t tile, int m, int c, int zform) {
  const int64_t total = (int64_t)m * c * npts;
  for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < total; t += (int64_t)gridDim.x * kBlock) {
    const int64_t p = t % npts;
    const int64_t ks = t / npts;
    const int s = (int)(ks % c);
    const int k = (int)(ks / c);
    const int64_t yi = ((p / tile) * m * c + ks) * tile + p % tile;
    double x = (double)Y[yi] + coef[kRowC * m + k] * X[s * stride + p];
    if (zform && Xm) x += coef[kRowBeta * m + k] * Xm[s * stride + p];
    out[ks * stride + p] = x;
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

// Points per lane: the requested width, else the widest one (FP64: 2, 16-byte mode accesses;
// FP32 modes: 4 in 2-D, 2 in 3-D, where 4 points of 6 components hold more registers than
// two waves per SIMD allow, and two waves of 2 points stream faster on MI355X than one of 4)
// for which every plane start and every group start is aligned to the vector size of each
// field (modes: V * sizeof(MT); the velocity gradient: V * sizeof(KT); the other fields,
// FP64: V * 8).
template <int D, typename MT, typename KT>
int pick_vec(const tfs_plan_s* p, const void* k0, const void* k1, const Levels& L, const void* tau,
             int max_v = 4) {
  const int widest = std::min(max_v, (sizeof(MT) == 4 && D == 2) ? 4 : 2);
  const int cand[3] = {widest, 2, 1};
  for (int V : cand) {
    if (V > widest) continue;
    if (p->vec_override && V != p->vec_override) continue;
    if (p->stride % V || p->tile % V) continue;
    const size_t bm = (size_t)V * sizeof(MT), bd = (size_t)V * 8, bk = (size_t)V * sizeof(KT);
    if (aligned(k0, bk) && aligned(k1, bk) && aligned(L.Xn, bd) && aligned(L.Xm, bd) && aligned(L.Xo, bd) &&
        aligned(L.Yn, bm) && aligned(L.Ym, bm) && aligned(L.Ym0, bm) && aligned(L.Yo, bm) && aligned(tau, bd) &&
        aligned(p->sp_rate, bd))
      return V;
  }
  return 1;
}

// Whole groups of V points with the V-wide kernel, the remaining npoints % V points with
// the V = 1 kernel; the diagnostics fold the block partials of both launches.
template <int D, typename MT, typename KT, int V, bool DIAG, bool SP, bool ZF>
hipError_t bdf2_launch(const tfs_plan_s* p, Bdf2Args<MT, KT> a, int64_t p_begin, int64_t ngroups, int part0,
                       int* nblocks) {
  a.p_begin = p_begin;
  a.ngroups = ngroups;
  a.part0 = part0;
  const int grid = grid_for(p, ngroups);
  hipLaunchKernelGGL((bdf2_kernel<D, MT, KT, V, DIAG, SP, false, ZF>), dim3(grid), dim3(kBlock), 0, p->stream, a);
  *nblocks = grid;
  return hipGetLastError();
}

template <int D, typename MT, typename KT, int V, bool DIAG, bool SP, bool ZF>
hipError_t bdf2_go_(const tfs_plan_s* p, const Bdf2Args<MT, KT>& a, double* diag_out) {
  const int64_t full = p->npoints / V, rest = p->npoints - full * V;
  int nb = 0, nt = 0;
  hipError_t e = hipSuccess;
  if (full > 0) e = bdf2_launch<D, MT, KT, V, DIAG, SP, ZF>(p, a, 0, full, 0, &nb);
  if (e == hipSuccess && rest > 0) e = bdf2_launch<D, MT, KT, 1, DIAG, SP, ZF>(p, a, full * V, rest, nb, &nt);
  if (e == hipSuccess && DIAG)
    hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(kBlock), 0, p->stream, a.part, nb + nt, diag_out);
  return e == hipSuccess ? hipGetLastError() : e;
}

// The spatial form reads FP64 velocity gradients only (an FP32-kappa plan refuses it).
template <int D, typename MT, typename KT, int V, bool ZF>
hipError_t bdf2_go_z(const tfs_plan_s* p, const Bdf2Args<MT, KT>& a, bool diag, double* diag_out) {
  if constexpr (sizeof(KT) == 8) {
    if (a.sp.rate || a.sp.src >= 0)
      return diag ? bdf2_go_<D, MT, KT, V, true, true, ZF>(p, a, diag_out)
                  : bdf2_go_<D, MT, KT, V, false, true, ZF>(p, a, diag_out);
  }
  return diag ? bdf2_go_<D, MT, KT, V, true, false, ZF>(p, a, diag_out)
              : bdf2_go_<D, MT, KT, V, false, false, ZF>(p, a, diag_out);
}

template <int D, typename MT, typename KT, int V>
hipError_t bdf2_go(const tfs_plan_s* p, const Bdf2Args<MT, KT>& a, bool diag, double* diag_out) {
  return p->zform ? bdf2_go_z<D, MT, KT, V, true>(p, a, diag, diag_out)
                  : bdf2_go_z<D, MT, KT, V, false>(p, a, diag, diag_out);
}

template <int D, typename MT, typename KT>
hipError_t bdf2_dispatch(const tfs_plan_s* p, int64_t n, const void* ka, const void* kb, const Levels& L,
                         double* tau, double* diag) {
  const int64_t st = p->stride;
  Bdf2Args<MT, KT> a;
  a.ka = static_cast<const KT*>(ka);
  a.kb = static_cast<const KT*>(kb);
  a.Xn = L.Xn;
  a.Xm = L.Xm;
  a.Xmm = p->zform ? L.Xmm : nullptr;
  a.Xo = L.Xo;
  a.Yn = static_cast<const MT*>(L.Yn);
  a.Ym = static_cast<const MT*>(L.Ym);
  a.Yo = static_cast<MT*>(L.Yo);
  a.tau = tau;
  a.coef = p->d_coef;
  a.part = L.part ? L.part : p->d_part;
  a.stride = st;
  a.tile = p->tile;
  a.m = p->m;
  a.s.a_diag = p->a_diag;
  a.sp.rate = p->sp_rate;
  a.sp.src = p->sp_source;
  a.s.eta = p->eta;
  a.s.s_ec = p->s_ec;
  a.s.inv_De = 1.0 / p->De;
  a.s.zeta = p->zeta[n + 1];
  a.s.tau_scale = p->tau_scale;
  int V = pick_vec<D, MT, KT>(p, ka, kb, L, tau);
  if (V > 1 && !aligned(a.Xmm, (size_t)V * 8)) V = 1;
  const bool dg = diag != nullptr;
  if constexpr (sizeof(MT) == 4) {
    if (V == 4) return bdf2_go<D, MT, KT, 4>(p, a, dg, diag);
  }
  if (V == 2) return bdf2_go<D, MT, KT, 2>(p, a, dg, diag);
  return bdf2_go<D, MT, KT, 1>(p, a, dg, diag);
}

template <int D, typename MT, typename KT, int V, bool DIAG, bool SP>
hipError_t start_launch(const tfs_plan_s* p, StartArgs<MT, KT> a, int64_t p_begin, int64_t ngroups, int part0,
                        int* nblocks) {
  a.p_begin = p_begin;
  a.ngroups = ngroups;
  a.part0 = part0;
  const int grid = grid_for(p, ngroups);
  hipLaunchKernelGGL((start_kernel<D, MT, KT, V, DIAG, SP>), dim3(grid), dim3(kBlock), 0, p->stream, a);
  *nblocks = grid;
  return hipGetLastError();
}

template <int D, typename MT, typename KT, int V, bool DIAG, bool SP>
hipError_t start_go_(const tfs_plan_s* p, const StartArgs<MT, KT>& a, double* diag_out) {
  const int64_t full = p->npoints / V, rest = p->npoints - full * V;
  int nb = 0, nt = 0;
  hipError_t e = hipSuccess;
  if (full > 0) e = start_launch<D, MT, KT, V, DIAG, SP>(p, a, 0, full, 0, &nb);
  if (e == hipSuccess && rest > 0) e = start_launch<D, MT, KT, 1, DIAG, SP>(p, a, full * V, rest, nb, &nt);
  if (e == hipSuccess && DIAG)
    hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(kBlock), 0, p->stream, a.part, nb + nt, diag_out);
  return e == hipSuccess ? hipGetLastError() : e;
}

template <int D, typename MT, typename KT, int V>
hipError_t start_go(const tfs_plan_s* p, const StartArgs<MT, KT>& a, bool diag, double* diag_out) {
  if constexpr (sizeof(KT) == 8) {
    if (a.sp.rate || a.sp.src >= 0)
      return diag ? start_go_<D, MT, KT, V, true, true>(p, a, diag_out)
                  : start_go_<D, MT, KT, V, false, true>(p, a, diag_out);
  }
  return diag ? start_go_<D, MT, KT, V, true, false>(p, a, diag_out)
              : start_go_<D, MT, KT, V, false, false>(p, a, diag_out);
}

// The split step (no local solve): a V-wide pass and a V = 1 tail pass, no diagnostics.
template <int D, typename MT, int V>
hipError_t bdf2_split_go(const tfs_plan_s* p, Bdf2Args<MT, double> a) {
  const int64_t full = p->npoints / V, rest = p->npoints - full * V;
  if (full > 0) {
    a.p_begin = 0;
    a.ngroups = full;
    a.part0 = 0;
    hipLaunchKernelGGL((bdf2_kernel<D, MT, double, V, false, false, true>), dim3(grid_for(p, full)), dim3(kBlock), 0,
                       p->stream, a);
  }
  if (rest > 0) {
    a.p_begin = full * V;
    a.ngroups = rest;
    a.part0 = 0;
    hipLaunchKernelGGL((bdf2_kernel<D, MT, double, 1, false, false, true>), dim3(grid_for(p, rest)), dim3(kBlock), 0,
                       p->stream, a);
  }
  return hipGetLastError();
}

template <int D, typename MT>
hipError_t bdf2_split_dispatch(const tfs_plan_s* p, int64_t n, const double* ka, const double* kb, const Levels& L,
                               double* G) {
  Bdf2Args<MT, double> a;
  a.ka = ka;
  a.kb = kb;
  a.Xn = L.Xn;
  a.Xm = L.Xm;
  a.Xmm = nullptr;
  a.Xo = L.Xo;
  a.Yn = static_cast<const MT*>(L.Yn);
  a.Ym = static_cast<const MT*>(L.Ym);
  a.Yo = static_cast<MT*>(L.Yo);
  a.tau = G;
  a.coef = p->d_coef;
  a.part = p->d_part;
  a.stride = p->stride;
  a.tile = p->tile;
  a.m = p->m;
  a.s.a_diag = p->a_diag;
  a.sp.rate = nullptr;
  a.sp.src = -1;
  a.s.eta = p->eta;
  a.s.s_ec = p->s_ec;
  a.s.inv_De = 1.0 / p->De;
  a.s.zeta = p->zeta[n + 1];
  a.s.tau_scale = p->tau_scale;
  const int V = pick_vec<D, MT, double>(p, ka, kb, L, G);
  if constexpr (sizeof(MT) == 4) {
    if (V == 4) return bdf2_split_go<D, MT, 4>(p, a);
  }
  if (V == 2) return bdf2_split_go<D, MT, 2>(p, a);
  return bdf2_split_go<D, MT, 1>(p, a);
}

template <int D, typename MT, typename KT>
hipError_t start_dispatch(const tfs_plan_s* p, const void* ka, const Levels& L, double* tau, double* diag) {
  StartArgs<MT, KT> a;
  a.ka = static_cast<const KT*>(ka);
  a.X0 = L.Xn;
  a.X1 = L.Xo;
  a.Y0 = static_cast<MT*>(L.Ym0);
  a.Y1 = static_cast<MT*>(L.Yo);
  a.tau = tau;
  a.coef = p->d_coef;
  a.part = L.part ? L.part : p->d_part;
  a.stride = p->stride;
  a.tile = p->tile;
  a.m = p->m;
  a.zform = p->zform ? 1 : 0;
  a.s.hgt = p->hg * p->theta;
  a.sp.rate = p->sp_rate;
  a.sp.src = p->sp_source;
  a.s.inv_De = 1.0 / p->De;
  a.s.src1 = p->hg * p->theta;
  a.s.sigma1 = p->sigma1;
  a.s.sigma2 = p->sigma2;
  a.s.gamma = p->gamma;
  a.s.theta = p->theta;
  a.s.hr = p->hr;
  const int V = pick_vec<D, MT, KT>(p, ka, nullptr, L, tau);
  const bool dg = diag != nullptr;
  if constexpr (sizeof(MT) == 4) {
    if (V == 4) return start_go<D, MT, KT, 4>(p, a, dg, diag);
  }
  if (V == 2) return start_go<D, MT, KT, 2>(p, a, dg, diag);
  return start_go<D, MT, KT, 1>(p, a, dg, diag);
}

template <int D, typename MT, typename KT, int V, bool DIAG, bool SP>
hipError_t exp_launch(const tfs_plan_s* p, ExpArgs<MT, KT> a, int64_t p_begin, int64_t ngroups, int part0,
                      int* nblocks) {
  a.p_begin = p_begin;
  a.ngroups = ngroups;
  a.part0 = part0;
  const int grid = grid_for(p, ngroups);
  hipLaunchKernelGGL((exp_kernel<D, MT, KT, V, DIAG, SP>), dim3(grid), dim3(kBlock), 0, p->stream, a);
  *nblocks = grid;
  return hipGetLastError();
}

template <int D, typename MT, typename KT, int V, bool DIAG, bool SP>
hipError_t exp_go_(const tfs_plan_s* p, const ExpArgs<MT, KT>& a, double* diag_out) {
  const int64_t full = p->npoints / V, rest = p->npoints - full * V;
  int nb = 0, nt = 0;
  hipError_t e = hipSuccess;
  if (full > 0) e = exp_launch<D, MT, KT, V, DIAG, SP>(p, a, 0, full, 0, &nb);
  if (e == hipSuccess && rest > 0) e = exp_launch<D, MT, KT, 1, DIAG, SP>(p, a, full * V, rest, nb, &nt);
  if (e == hipSuccess && DIAG)
    hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(kBlock), 0, p->stream, a.part, nb + nt, diag_out);
  return e == hipSuccess ? hipGetLastError() : e;
}

template <int D, typename MT, typename KT, bool SP>
hipError_t exp_go(const tfs_plan_s* p, const ExpArgs<MT, KT>& a, int V, double* diag) {
  if constexpr (sizeof(MT) == 4 && D == 2) {
    if (V == 4)
      return diag ? exp_go_<D, MT, KT, 4, true, SP>(p, a, diag) : exp_go_<D, MT, KT, 4, false, SP>(p, a, diag);
  }
  if (V == 2) return diag ? exp_go_<D, MT, KT, 2, true, SP>(p, a, diag) : exp_go_<D, MT, KT, 2, false, SP>(p, a, diag);
  return diag ? exp_go_<D, MT, KT, 1, true, SP>(p, a, diag) : exp_go_<D, MT, KT, 1, false, SP>(p, a, diag);
}

template <int D, typename MT, typename KT>
hipError_t exp_dispatch(const tfs_plan_s* p, int64_t n, const void* ka, const void* kb, const Levels& L,
                        double* tau, double* diag) {
  ExpArgs<MT, KT> a;
  a.ka = static_cast<const KT*>(ka);
  a.kb = (n >= 1) ? static_cast<const KT*>(kb) : nullptr;
  a.Xn = L.Xn;
  a.Xo = L.Xo;
  a.Yn = static_cast<const MT*>(L.Yn);
  a.Yo = static_cast<MT*>(L.Yo);
  a.tau = tau;
  a.Hout = nullptr;
  a.coef = p->d_coef;
  a.part = L.part ? L.part : p->d_part;
  a.stride = p->stride;
  a.tile = p->tile;
  a.m = p->m;
  a.s.a_diag = 1.0 + p->q_e / p->De;
  a.sp.rate = p->sp_rate;
  a.sp.src = p->sp_source;
  a.s.q = p->q_e;
  a.s.s_h = p->s_h;
  a.s.inv_De = 1.0 / p->De;
  a.s.zeta = p->zeta[n + 1];
  a.s.tau_scale = p->tau_scale;
  a.s.eta_e = p->eta_e;
  a.s.fa = 1.5;
  a.s.fb = -0.5;
  a.s.first = n == 0 ? 1 : 0;
  // the level-n modes are read (not at n = 0) and written: both alignments matter
  Levels A = L;
  A.Ym = nullptr;
  // two compensated sums per component: in 3-D four points per lane would spill
  const int V = pick_vec<D, MT, KT>(p, ka, a.kb, A, tau, D == 3 ? 2 : 4);
  if constexpr (sizeof(KT) == 8) {
    if (a.sp.rate || a.sp.src >= 0) return exp_go<D, MT, KT, true>(p, a, V, diag);
  }
  return exp_go<D, MT, KT, false>(p, a, V, diag);
}

// The split exponential step (no local solve): a V-wide pass and a V = 1 tail pass.
template <int D, typename MT, int V>
hipError_t exp_split_go(const tfs_plan_s* p, ExpArgs<MT, double> a) {
  const int64_t full = p->npoints / V, rest = p->npoints - full * V;
  a.part0 = 0;
  if (full > 0) {
    a.p_begin = 0;
    a.ngroups = full;
    hipLaunchKernelGGL((exp_kernel<D, MT, double, V, false, false, true>), dim3(grid_for(p, full)), dim3(kBlock), 0,
                       p->stream, a);
  }
  if (rest > 0) {
    a.p_begin = full * V;
    a.ngroups = rest;
    hipLaunchKernelGGL((exp_kernel<D, MT, double, 1, false, false, true>), dim3(grid_for(p, rest)), dim3(kBlock), 0,
                       p->stream, a);
  }
  return hipGetLastError();
}

template <int D, typename MT>
hipError_t exp_split_dispatch(const tfs_plan_s* p, int64_t n, const double* ka, const double* kb, const Levels& L,
                              double* G, double* H) {
  ExpArgs<MT, double> a;
  a.ka = ka;
  a.kb = (n >= 1) ? kb : nullptr;
  a.Xn = L.Xn;
  a.Xo = L.Xo;
  a.Yn = static_cast<const MT*>(L.Yn);
  a.Yo = static_cast<MT*>(L.Yo);
  a.tau = G;
  a.Hout = H;
  a.coef = p->d_coef;
  a.part = nullptr;
  a.stride = p->stride;
  a.tile = p->tile;
  a.m = p->m;
  a.s.a_diag = 1.0 + p->q_e / p->De;
  a.sp.rate = nullptr;
  a.sp.src = -1;
  a.s.q = p->q_e;
  a.s.s_h = p->s_h;
  a.s.inv_De = 1.0 / p->De;
  a.s.zeta = p->zeta[n + 1];
  a.s.tau_scale = p->tau_scale;
  a.s.eta_e = p->eta_e;
  a.s.fa = 1.5;
  a.s.fb = -0.5;
  a.s.first = n == 0 ? 1 : 0;
  Levels A = L;
  A.Ym = nullptr;
  int V = pick_vec<D, MT, double>(p, ka, a.kb, A, G, D == 3 ? 2 : 4);
  if (!aligned(H, (size_t)V * 8)) V = 1;
  if constexpr (sizeof(MT) == 4 && D == 2) {
    if (V == 4) return exp_split_go<D, MT, 4>(p, a);
  }
  if (V == 2) return exp_split_go<D, MT, 2>(p, a);
  return exp_split_go<D, MT, 1>(p, a);
}

}  // namespace

// a V-wide pass and a V = 1 tail pass
int max_blocks(const tfs_plan_s* p) { return 2 * p->num_cus * kMaxBlocksPerCU; }

// Static scratch of tfs_step_noalloc: the diagnostics block partials of one step (the V-wide
// pass and the tail pass of a 256-CU device at the default 16 blocks per CU), 384 KiB.  Every
// device holds its own copy until the process ends.  Host code never passes the symbol itself
// to a kernel or a copy: only the address scratch_address returns for the device.
static __device__ __align__(256) double scratch[(size_t)kScratchPartials * kNumDiag];

hipError_t scratch_address(int device, double** out) {
  static std::mutex mu;
  static std::vector<double*> cache;
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((size_t)device < cache.size() && cache[device]) {
    *out = cache[device];
    return hipSuccess;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if ((size_t)device >= cache.size()) cache.resize((size_t)device + 1, nullptr);
  cache[device] = static_cast<double*>(ptr);
  *out = cache[device];
  return hipSuccess;
}

// The plan's (dim, mode precision, kappa precision) instance of a dispatcher; FP32 velocity
// gradients exist only with FP32 modes.
#define TFS_DISPATCH(fn, ...)                                                                      \
  (p->precision == TFS_FP64                                                                        \
       ? (p->d == 2 ? fn<2, double, double>(__VA_ARGS__) : fn<3, double, double>(__VA_ARGS__))    \
       : p->kappa_f32                                                                              \
             ? (p->d == 2 ? fn<2, float, float>(__VA_ARGS__) : fn<3, float, float>(__VA_ARGS__))  \
             : (p->d == 2 ? fn<2, float, double>(__VA_ARGS__) : fn<3, float, double>(__VA_ARGS__)))

hipError_t launch_bdf2(const tfs_plan_s* p, int64_t n, const void* ka, const void* kb, const Levels& L,
                       double* tau, double* diag) {
  if (p->npoints == 0) {
    if (diag) hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(kBlock), 0, p->stream, p->d_part, 0, diag);
    return hipGetLastError();
  }
  return TFS_DISPATCH(bdf2_dispatch, p, n, ka, kb, L, tau, diag);
}

hipError_t launch_bdf2_split(const tfs_plan_s* p, int64_t n, const double* ka, const double* kb, const Levels& L,
                             double* G) {
  if (p->npoints == 0) return hipSuccess;
  if (p->precision == TFS_FP64)
    return p->d == 2 ? bdf2_split_dispatch<2, double>(p, n, ka, kb, L, G)
                     : bdf2_split_dispatch<3, double>(p, n, ka, kb, L, G);
  return p->d == 2 ? bdf2_split_dispatch<2, float>(p, n, ka, kb, L, G)
                   : bdf2_split_dispatch<3, float>(p, n, ka, kb, L, G);
}

hipError_t launch_startup(const tfs_plan_s* p, const void* ka, const Levels& L, double* tau, double* diag) {
  if (p->npoints == 0) {
    if (diag) hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(kBlock), 0, p->stream, p->d_part, 0, diag);
    return hipGetLastError();
  }
  return TFS_DISPATCH(start_dispatch, p, ka, L, tau, diag);
}

hipError_t launch_exp(const tfs_plan_s* p, int64_t n, const void* ka, const void* kb, const Levels& L,
                      double* tau, double* diag) {
  if (p->npoints == 0) {
    if (diag) hipLaunchKernelGGL(diag_finish_kernel, dim3(1), dim3(kBlock), 0, p->stream, p->d_part, 0, diag);
    return hipGetLastError();
  }
  return TFS_DISPATCH(exp_dispatch, p, n, ka, kb, L, tau, diag);
}

hipError_t launch_exp_split(const tfs_plan_s* p, int64_t n, const double* ka, const double* kb, const Levels& L,
                            double* G, double* H) {
  if (p->npoints == 0) return hipSuccess;
  if (p->precision == TFS_FP64)
    return p->d == 2 ? exp_split_dispatch<2, double>(p, n, ka, kb, L, G, H)
                     : exp_split_dispatch<3, double>(p, n, ka, kb, L, G, H);
  return p->d == 2 ? exp_split_dispatch<2, float>(p, n, ka, kb, L, G, H)
                   : exp_split_dispatch<3, float>(p, n, ka, kb, L, G, H);
}

hipError_t launch_modes_to_plain(const tfs_plan_s* p, int64_t level, const double* X, const void* Y, double* Xk) {
  if (p->npoints == 0) return hipSuccess;
  const int64_t st = p->stride, xs = (int64_t)p->c * st;
  const double* Xs = X + (level % p->xlev) * xs;
  const double* Xm = (p->zform && level >= 1) ? X + ((level - 1) % p->xlev) * xs : nullptr;
  const int slot = p->scheme == TFS_SCHEME_EXP ? 0 : (int)(level % 2);   // the exponential scheme keeps one level
  const int64_t total = (int64_t)p->m * p->c * p->npoints;
  int grid = (int)((total + kBlock - 1) / kBlock);
  if (grid > 65536) grid = 65536;
  const int zf = p->zform ? 1 : 0;
  if (p->precision == TFS_FP64) {
    const double* Ys = static_cast<const double*>(Y) + (int64_t)slot * p->m * p->c * st;
    hipLaunchKernelGGL(plain_kernel<double>, dim3(grid), dim3(kBlock), 0, p->stream, Xs, Xm, Ys, p->d_coef, Xk,
                       p->npoints, st, p->tile, p->m, p->c, zf);
  } else {
    const float* Ys = static_cast<const float*>(Y) + (int64_t)slot * p->m * p->c * st;
    hipLaunchKernelGGL(plain_kernel<float>, dim3(grid), dim3(kBlock), 0, p->stream, Xs, Xm, Ys, p->d_coef, Xk,
                       p->npoints, st, p->tile, p->m, p->c, zf);
  }
  return hipGetLastError();
}

}  // namespace tfs

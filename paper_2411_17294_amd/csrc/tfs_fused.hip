// Temporally fused exponential-mode steps for an analytic velocity gradient.
//
// When kappa(x, t) is a closed-form field (a sum of Fourier terms,
//   kappa_ij(x, t) = sum_n B_n,ij sin(k_n . x + phi_n + omega_n t)  on [0, 2 pi)^d),
// no caller interaction is needed between steps: one launch advances every point through
// K time levels of the exponential-mode scheme (the per-point arithmetic of exp_group,
// V = 1) with the point's whole state in registers.  The mode level (m c values), X and
// the previous kappa stay on chip for all K steps; HBM is read once at the start and
// written once at the end, so the launch is bound by arithmetic, not by memory.
//
// Per point and step: kappa at t_n evaluated from the field (FP64 sine per term), the
// half-step gradient kappa~ = 3/2 kappa^n - 1/2 kappa^{n-1} (kappa^0 at n = 0), the mode
// update Y_k <- e_k Y_k + f_k X with H and (compensated) G, the c x c solve and, at the last
// step, tau.  The mode count is a template parameter so the mode array lives in registers.
#include "tfs_device.h"
#include "tfs_internal.h"

namespace tfs {
namespace {

using namespace dev;

constexpr int kFusedBlock = 128;
// A time-varying field's terms are advanced by angle addition with their (sin, cos) in LDS
// when a lane has at most this many of them (kRotTerms * 16 B * kFusedBlock per block); more
// terms are evaluated with one sincos each per step.
constexpr int kRotTerms = 64;
// Steps between fresh sincos evaluations of the rotated terms (bounds the drift of the
// repeated rotation to a few tens of rounding errors).
constexpr int kReseed = 32;
// Largest field table (bytes) copied into each block's LDS.
constexpr size_t kTabLdsMax = 32768;
// Doubles of padding per row of the LDS copy: a 3-D row is 16 doubles, 128 bytes, so the rows
// that the lanes of a point read at once (consecutive terms) would all start on the same LDS
// bank; 16 bytes more per row spreads four of them over distinct banks.
constexpr int kTabPad = 2;

template <typename MT>
struct FusedArgs {
  double* X;              // ring [2][c][stride]: level n0 in slot n0 % 2
  MT* Y;                  // one mode level (tiled), updated in place
  double* tau;            // [c][stride] or null (level n0 + nsteps)
  const double* coef;     // [kNumCoefAll][m], ExpRow order
  const double* zeta;     // [max_steps + 1] mass-mode increments
  const double* field;    // [nterms][d + 4 + d*d]: k_n, phi_n, omega_n, cos/sin(omega_n dt), B_n
  int64_t npoints, stride, tile, n0, nsteps, grid, point0;
  int nterms, steady;
  double dt, a_diag, q, s_h, inv_De, tau_scale, eta_e, fa, fb;
  double eta, s_ec;       // BDF2: eta = sum_k b0 c_k, s_ec = sum_k eta_k c_k
};

// v moved within each quad of lanes by the DPP quad permutation CTRL.
template <int CTRL>
__device__ __forceinline__ double quad_mov(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over the L lanes of a point (L = 1, 2 or 4 consecutive lanes); every lane gets the
// same value: pairs exchange by quad_perm [1, 0, 3, 2], then halves of the quad by
// [2, 3, 0, 1].
template <int L>
__device__ __forceinline__ double lanes_sum(double v) {
  if constexpr (L >= 2) v = v + quad_mov<0xB1>(v);
  if constexpr (L == 4) v = v + quad_mov<0x4E>(v);
  return v;
}

// The velocity gradient driving a step at the point x: kappa(t) when gb = 0, or the
// half-step extrapolation ga kappa(t) + gb kappa(t - dt) (row-major d x d).  The earlier
// sine comes from the later one by angle addition, sin(a - w dt) = sin a cos(w dt) -
// cos a sin(w dt), so each term costs one sincos.  Lane h of the point's L lanes sums the
// terms n = h, h + L, ...; the caller adds the lanes' sums.
// The field table is read from LDS (a block copy of it, rows padded by kTabPad) or from
// global memory: the lanes of a point read different terms, so global reads are vector
// loads, one memory round trip per term.  f(n, j): entry j of term n's row.
template <bool LF, int W>
struct FieldTab {
  const double* t;                                   // LDS copy (LF) or global table
  __device__ __forceinline__ double operator()(int n, int j) const {
    if constexpr (LF) return t[n * (W + kTabPad) + j];
    else return load_uniform(opaque_ptr(t) + n * W + j);
  }
};

template <int D, int L, typename FT>
__device__ __forceinline__ void field_kappa(const FT& f, int nterms, int h, const double (&x)[D], double t,
                                            double ga, double gb, double (&kap)[D * D]) {
  constexpr int W = D + 4 + D * D;
#pragma unroll
  for (int q = 0; q < D * D; ++q) kap[q] = 0.0;
  for (int n = h; n < nterms; n += L) {
    double th = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) th += x[j] * f(n, j);
    th = th + f(n, D) + f(n, D + 1) * t;
    double sn, cn;
    sincos(th, &sn, &cn);
    double wgt = sn;
    if (gb != 0.0) wgt = ga * sn + gb * (sn * f(n, D + 2) - cn * f(n, D + 3));
#pragma unroll
    for (int q = 0; q < D * D; ++q) kap[q] += wgt * f(n, D + 4 + q);
  }
#pragma unroll
  for (int q = 0; q < D * D; ++q) kap[q] = lanes_sum<L>(kap[q]);
}

// (sin, cos) of the lane's terms at time t into LDS (rot[i * kFusedBlock + lane]).
template <int D, int L, typename FT>
__device__ __forceinline__ void rot_seed(const FT& f, int nterms, int h, const double (&x)[D], double t,
                                         double2* rot) {
  constexpr int W = D + 4 + D * D;
  int i = 0;
  for (int n = h; n < nterms; n += L, ++i) {
    double th = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) th += x[j] * f(n, j);
    th = th + f(n, D) + f(n, D + 1) * t;
    double sn, cn;
    sincos(th, &sn, &cn);
    rot[i * kFusedBlock + threadIdx.x] = make_double2(sn, cn);
  }
}

// kappa~ from the lane's rotated terms (their sin and cos at t_n), as field_kappa; then the
// terms move to t_{n+1} by angle addition (the caller re-seeds them every kReseed steps).
template <int D, int L, typename FT>
__device__ __forceinline__ void rot_kappa(const FT& f, int nterms, int h, double ga, double gb, double2* rot,
                                          double (&kap)[D * D]) {
  constexpr int W = D + 4 + D * D;
#pragma unroll
  for (int q = 0; q < D * D; ++q) kap[q] = 0.0;
  const int cnt = (nterms - h + L - 1) / L;
  if constexpr (D == 3) {
    // 3-D: term i + 1's reads are issued before term i's arithmetic (two register sets, the
    // loop unrolled by two so that they alternate without copies).  Left to itself the
    // scheduler interleaved reads and uses in the BDF2 kernel, one LDS round trip per read.
    struct Term { double2 sc; double cw, sw, b[D * D]; };
    auto read = [&](int i, Term& t) {
      const int n = h + i * L;
      t.sc = rot[i * kFusedBlock + threadIdx.x];
      t.cw = f(n, D + 2);
      t.sw = f(n, D + 3);
#pragma unroll
      for (int q = 0; q < D * D; ++q) t.b[q] = f(n, D + 4 + q);
    };
    auto use = [&](int i, const Term& t) {
      double wgt = t.sc.x;
      if (gb != 0.0) wgt = ga * t.sc.x + gb * (t.sc.x * t.cw - t.sc.y * t.sw);
#pragma unroll
      for (int q = 0; q < D * D; ++q) kap[q] += wgt * t.b[q];
      rot[i * kFusedBlock + threadIdx.x] =
          make_double2(t.sc.x * t.cw + t.sc.y * t.sw, t.sc.y * t.cw - t.sc.x * t.sw);
    };
    if (cnt > 0) {
      Term A, B;
      read(0, A);
      for (int i = 0; i < cnt; i += 2) {
        read(min(i + 1, cnt - 1), B);      // (past the last term: a re-read, unused)
        __builtin_amdgcn_sched_barrier(0);
        use(i, A);
        if (i + 1 < cnt) {
          read(min(i + 2, cnt - 1), A);
          __builtin_amdgcn_sched_barrier(0);
          use(i + 1, B);
        }
      }
    }
  } else {
    // 2-D: two terms in flight (measured faster than one)
#pragma unroll 2
    for (int i = 0; i < cnt; ++i) {
      const int n = h + i * L;
      const double2 sc = rot[i * kFusedBlock + threadIdx.x];
      const double cw = f(n, D + 2), sw = f(n, D + 3);
      double wgt = sc.x;
      if (gb != 0.0) wgt = ga * sc.x + gb * (sc.x * cw - sc.y * sw);
#pragma unroll
      for (int q = 0; q < D * D; ++q) kap[q] += wgt * f(n, D + 4 + q);
      rot[i * kFusedBlock + threadIdx.x] = make_double2(sc.x * cw + sc.y * sw, sc.y * cw - sc.x * sw);
    }
  }
#pragma unroll
  for (int q = 0; q < D * D; ++q) kap[q] = lanes_sum<L>(kap[q]);
}

// The lane's modes advanced one step: Y_k <- e_k Y_k + f_k X (Y_k = -q_k X before the first
// step), with H = sum (1 - e_k) Y_k and G = sum lambda_k dt Y_k^{new} (compensated).
template <int C, typename MT, int M, int MH, bool FIRST>
__device__ __forceinline__ void mode_pass(const double* coef, int k0, const double (&X)[C], MT (&y)[MH][C],
                                          double (&H)[C], double (&Gs)[C], double (&Ge)[C]) {
#pragma unroll
  for (int s = 0; s < C; ++s) { H[s] = 0.0; Gs[s] = 0.0; Ge[s] = 0.0; }
  // the coefficients are read again every step (scalar-cache hits) instead of holding 5 M
  // of them in scalar registers across the step loop
  const double* cf = opaque_ptr(coef) + k0;
#pragma unroll
  for (int kk = 0; kk < MH; ++kk) {
    const double ek = load_uniform(cf + kRowE * M + kk);
    const double fk = load_uniform(cf + kRowF * M + kk);
    const double lk = load_uniform(cf + kRowLdt * M + kk);
    const double ok = load_uniform(cf + kRowOneME * M + kk);
    double qk = 0.0;
    if constexpr (FIRST) qk = load_uniform(cf + kRowQ * M + kk);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const double yv = FIRST ? -qk * X[s] : (double)y[kk][s];
      const MT out = (MT)(ek * yv + fk * X[s]);
      y[kk][s] = out;
      H[s] += ok * yv;
      two_sum_acc(Gs[s], Ge[s], mul_rn(lk, (double)out));
    }
    // keep each mode's coefficients local to its iteration: hoisting all of them to the
    // top of the step exhausts the scalar registers
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Dynamic LDS of a fused launch: the field table (when it is copied, nterms rows of W +
// kTabPad doubles), then the rotated terms.  Every thread of the block takes part in the
// copy, before any returns.
template <int D, bool LF, typename MT>
__device__ __forceinline__ FieldTab<LF, D + 4 + D * D> stage_field(const FusedArgs<MT>& a, double2* smem,
                                                                   double2** rot) {
  constexpr int W = D + 4 + D * D;
  FieldTab<LF, W> f;
  if constexpr (LF) {
    const int tabn = a.nterms * W;
    double* tab = reinterpret_cast<double*>(smem);
    for (int i = threadIdx.x; i < tabn; i += kFusedBlock) tab[(i / W) * (W + kTabPad) + i % W] = a.field[i];
    __syncthreads();
    *rot = smem + (a.nterms * (W + kTabPad) + 1) / 2;
    f.t = tab;
  } else {
    *rot = smem;
    f.t = a.field;
  }
  return f;
}

// One point per L consecutive lanes; lane h of them holds modes [h M/L, (h+1) M/L) in
// registers.  The lanes add their partial mode sums (H, G) and field terms, then both run
// the point's c x c solve on the same values.
template <int D, typename MT, int M, int L, bool LF>
__global__ __launch_bounds__(kFusedBlock) void fused_exp_kernel(const FusedArgs<MT> a) {
  constexpr int C = Sym<D>::C;
  constexpr int MH = M / L;
  const int64_t g = (int64_t)blockIdx.x * kFusedBlock + threadIdx.x;
  const int64_t p = g / L;
  const int h = (int)(g % L);
  extern __shared__ double2 smem[];
  double2* rot;
  const auto f = stage_field<D, LF>(a, smem, &rot);
  if (p >= a.npoints) return;
  const int64_t st = a.stride, T = a.tile;
  const int64_t ym = (p / T) * (int64_t)M * C * T + p % T;   // mode (0, 0) of the point
  const int k0 = h * MH;

  double x[D];
  {
    int64_t r = a.point0 + p;
    const double hx = 2.0 * 3.14159265358979323846 / (double)a.grid;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      x[j] = hx * (double)(r % a.grid);
      r /= a.grid;
    }
  }
  double X[C];
  const int64_t s0 = a.n0 % 2;
#pragma unroll
  for (int s = 0; s < C; ++s) X[s] = a.X[(s0 * C + s) * st + p];
  MT y[MH][C];
  if (a.n0 > 0) {
#pragma unroll
    for (int k = 0; k < MH; ++k)
#pragma unroll
      for (int s = 0; s < C; ++s) y[k][s] = a.Y[ym + (int64_t)((k0 + k) * C + s) * T];
  }
  // a steady field is evaluated once; a time-varying one is rotated in LDS when it fits
  const bool rotate = !a.steady && (a.nterms + L - 1) / L <= kRotTerms;
  double ks[D * D];
  if (a.steady) field_kappa<D, L>(f, a.nterms, h, x, 0.0, 1.0, 0.0, ks);
  if (rotate) rot_seed<D, L>(f, a.nterms, h, x, (double)a.n0 * a.dt, rot);
  const int64_t sn = (a.n0 + a.nsteps) % 2;
  double tout[C];
#pragma unroll
  for (int s = 0; s < C; ++s) tout[s] = 0.0;

  for (int64_t j = 0; j < a.nsteps; ++j) {
    const int64_t n = a.n0 + j;
    const bool first = n == 0;
    if (j + 1 == a.nsteps && h == 0) {
      // level n0 + nsteps - 1 goes to the other slot of the ring
#pragma unroll
      for (int s = 0; s < C; ++s) a.X[((1 - sn) * C + s) * st + p] = X[s];
    }
    double k[D * D];
    if (a.steady) {
#pragma unroll
      for (int q = 0; q < D * D; ++q) k[q] = first ? ks[q] : a.fa * ks[q] + a.fb * ks[q];
    } else if (rotate) {
      rot_kappa<D, L>(f, a.nterms, h, a.fa, first ? 0.0 : a.fb, rot, k);
      if ((j + 1) % kReseed == 0) rot_seed<D, L>(f, a.nterms, h, x, (double)(n + 1) * a.dt, rot);
    } else if (first) {
      field_kappa<D, L>(f, a.nterms, h, x, 0.0, 1.0, 0.0, k);
    } else {
      field_kappa<D, L>(f, a.nterms, h, x, (double)n * a.dt, a.fa, a.fb, k);
    }

    double H[C], Gs[C], Ge[C];
    if (first) mode_pass<C, MT, M, MH, true>(a.coef, k0, X, y, H, Gs, Ge);
    else mode_pass<C, MT, M, MH, false>(a.coef, k0, X, y, H, Gs, Ge);
    double Hv[C], AH[C], R[C], G[C];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      Hv[s] = lanes_sum<L>(H[s]) + a.s_h * X[s];
      G[s] = lanes_sum<L>(Gs[s] + Ge[s]);
    }
    apply_K<D>(k, Hv, AH);
    const double zeta = a.zeta[n + 1];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const int i = Sym<D>::i(s), jj = Sym<D>::j(s);
      const double S = k[i * D + jj] + k[jj * D + i];
      R[s] = X[s] - (AH[s] - a.inv_De * Hv[s]) + zeta * S;
    }
    double Mx[C][C];
    build_M<D>(k, a.a_diag, a.q, Mx);
    solve_pivot<C>(Mx, R);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      tout[s] = a.tau_scale * (a.eta_e * R[s] - G[s]);
      X[s] = R[s];
    }
  }

  if (h == 0) {
#pragma unroll
    for (int s = 0; s < C; ++s) {
      a.X[(sn * C + s) * st + p] = X[s];
      if (a.tau) a.tau[s * st + p] = tout[s];
    }
  }
#pragma unroll
  for (int k = 0; k < MH; ++k)
#pragma unroll
    for (int s = 0; s < C; ++s) a.Y[ym + (int64_t)((k0 + k) * C + s) * T] = y[k][s];
}

// One BDF2 step of the lane's modes (Sec. 4.1 in the representation Y_k = X_k - c_k X):
// h_k = 2 Y_k^n - Y_k^{n-1}/2, Y_k^{n+1} = d_k h_k + d_k c_k P written over Y_k^{n-1}, and
// the lane's part of G = sum eta_k h_k (compensated).
template <int C, typename MT, int M, int MH>
__device__ __forceinline__ void bdf2_mode_pass(const double* coef, int k0, const double (&P)[C],
                                               const MT (&yn)[MH][C], MT (&ym)[MH][C], double (&Gs)[C],
                                               double (&Ge)[C]) {
#pragma unroll
  for (int s = 0; s < C; ++s) { Gs[s] = 0.0; Ge[s] = 0.0; }
  const double* cf = opaque_ptr(coef) + k0;
#pragma unroll
  for (int kk = 0; kk < MH; ++kk) {
    const double dk = load_uniform(cf + kRowD * M + kk);
    const double dck = load_uniform(cf + kRowDC * M + kk);
    const double ek = load_uniform(cf + kRowEta * M + kk);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const double h = 2.0 * (double)yn[kk][s] - 0.5 * (double)ym[kk][s];
      ym[kk][s] = (MT)(dk * h + dck * P[s]);
      two_sum_acc(Gs[s], Ge[s], mul_rn(ek, h));
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// One fused BDF2 time level n -> n+1 of a point: kappa~ = 2 kappa(t_n) - kappa(t_{n-1}) from
// the field, the modes (yn = level n, ym = level n-1, overwritten with n+1), the c x c solve.
template <int D, typename MT, int M, int L, typename FT>
__device__ __forceinline__ void bdf2_fused_step(const FusedArgs<MT>& a, const FT& f, int h, int64_t n, int64_t j,
                                                bool rotate, const double (&x)[D], const double (&ks)[D * D], double2* rot,
                                                double (&Xn)[Sym<D>::C], double (&Xm)[Sym<D>::C],
                                                const MT (&yn)[M / L][Sym<D>::C], MT (&ym)[M / L][Sym<D>::C],
                                                double (&tout)[Sym<D>::C]) {
  constexpr int C = Sym<D>::C;
  double k[D * D];
  if (a.steady) {
#pragma unroll
    for (int q = 0; q < D * D; ++q) k[q] = 2.0 * ks[q] - ks[q];
  } else if (rotate) {
    rot_kappa<D, L>(f, a.nterms, h, 2.0, -1.0, rot, k);
    if ((j + 1) % kReseed == 0) rot_seed<D, L>(f, a.nterms, h, x, (double)(n + 1) * a.dt, rot);
  } else {
    field_kappa<D, L>(f, a.nterms, h, x, (double)n * a.dt, 2.0, -1.0, k);
  }
  double P[C], Gs[C], Ge[C], G[C], AG[C], R[C];
#pragma unroll
  for (int s = 0; s < C; ++s) P[s] = 2.0 * Xn[s] - 0.5 * Xm[s];
  bdf2_mode_pass<C, MT, M, M / L>(a.coef, h * (M / L), P, yn, ym, Gs, Ge);
#pragma unroll
  for (int s = 0; s < C; ++s) G[s] = lanes_sum<L>(Gs[s] + Ge[s]) + a.s_ec * P[s];
  apply_K<D>(k, G, AG);
  const double zeta = a.zeta[n + 1];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    const int i = Sym<D>::i(s), jj = Sym<D>::j(s);
    const double S = k[i * D + jj] + k[jj * D + i];
    R[s] = P[s] - (AG[s] - a.inv_De * G[s]) + zeta * S;
  }
  double Mx[C][C];
  build_M<D>(k, a.a_diag, a.eta, Mx);
  solve_pivot<C>(Mx, R);
#pragma unroll
  for (int s = 0; s < C; ++s) {
    tout[s] = a.tau_scale * (a.eta * R[s] - G[s]);
    Xm[s] = Xn[s];
    Xn[s] = R[s];
  }
}

// Fused BDF2 levels n0 -> n0 + nsteps (n0 >= 1): L lanes per point, each with its share of
// both mode levels in registers; level j returns to ring slot j % 2.
template <int D, typename MT, int M, int L, bool LF>
__global__ __launch_bounds__(kFusedBlock) void fused_bdf2_kernel(const FusedArgs<MT> a) {
  constexpr int C = Sym<D>::C;
  constexpr int MH = M / L;
  const int64_t g = (int64_t)blockIdx.x * kFusedBlock + threadIdx.x;
  const int64_t p = g / L;
  const int h = (int)(g % L);
  extern __shared__ double2 smem[];
  double2* rot;
  const auto f = stage_field<D, LF>(a, smem, &rot);
  if (p >= a.npoints) return;
  const int64_t st = a.stride, T = a.tile;
  const int64_t ys = (int64_t)M * C * st;                     // one ring slot
  const int64_t ym0 = (p / T) * (int64_t)M * C * T + p % T;
  const int k0 = h * MH;
  double x[D];
  {
    int64_t r = a.point0 + p;
    const double hx = 2.0 * 3.14159265358979323846 / (double)a.grid;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      x[j] = hx * (double)(r % a.grid);
      r /= a.grid;
    }
  }
  const int64_t sa = a.n0 % 2, sb = 1 - sa;
  double Xn[C], Xm[C], tout[C];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    Xn[s] = a.X[(sa * C + s) * st + p];
    Xm[s] = a.X[(sb * C + s) * st + p];
    tout[s] = 0.0;
  }
  MT ya[MH][C], yb[MH][C];
#pragma unroll
  for (int k = 0; k < MH; ++k)
#pragma unroll
    for (int s = 0; s < C; ++s) {
      ya[k][s] = a.Y[sa * ys + ym0 + (int64_t)((k0 + k) * C + s) * T];
      yb[k][s] = a.Y[sb * ys + ym0 + (int64_t)((k0 + k) * C + s) * T];
    }
  const bool rotate = !a.steady && (a.nterms + L - 1) / L <= kRotTerms;
  double ks[D * D];
  if (a.steady) field_kappa<D, L>(f, a.nterms, h, x, 0.0, 1.0, 0.0, ks);
  if (rotate) rot_seed<D, L>(f, a.nterms, h, x, (double)a.n0 * a.dt, rot);
  // ya holds level n and yb level n - 1; the step overwrites yb with n + 1, then the two swap
  // (register moves: calling the step with the roles exchanged every other step holds more
  // registers)
  for (int64_t j = 0; j < a.nsteps; ++j) {
    bdf2_fused_step<D, MT, M, L>(a, f, h, a.n0 + j, j, rotate, x, ks, rot, Xn, Xm, ya, yb, tout);
#pragma unroll
    for (int k = 0; k < MH; ++k)
#pragma unroll
      for (int s = 0; s < C; ++s) {
        const MT t = ya[k][s];
        ya[k][s] = yb[k][s];
        yb[k][s] = t;
      }
  }
  // after the loop ya holds level n0 + nsteps and yb level n0 + nsteps - 1
  const int64_t sn = (a.n0 + a.nsteps) % 2;
  if (h == 0) {
#pragma unroll
    for (int s = 0; s < C; ++s) {
      a.X[(sn * C + s) * st + p] = Xn[s];
      a.X[((1 - sn) * C + s) * st + p] = Xm[s];
      if (a.tau) a.tau[s * st + p] = tout[s];
    }
  }
#pragma unroll
  for (int k = 0; k < MH; ++k)
#pragma unroll
    for (int s = 0; s < C; ++s) {
      a.Y[sn * ys + ym0 + (int64_t)((k0 + k) * C + s) * T] = ya[k][s];
      a.Y[(1 - sn) * ys + ym0 + (int64_t)((k0 + k) * C + s) * T] = yb[k][s];
    }
}

template <int D, typename MT, int M, int L, bool BDF2>
hipError_t fused_go(const tfs_plan_s* p, int64_t n0, int64_t nsteps, double* X, void* Y, double* tau) {
  FusedArgs<MT> a;
  a.X = X;
  a.Y = static_cast<MT*>(Y);
  a.tau = tau;
  a.coef = p->d_coef;
  a.zeta = p->d_zeta;
  a.field = p->d_field;
  a.npoints = p->npoints;
  a.stride = p->stride;
  a.tile = p->tile;
  a.n0 = n0;
  a.nsteps = nsteps;
  a.grid = p->field_grid;
  a.point0 = p->field_point0;
  a.nterms = p->field_terms;
  a.steady = p->field_steady ? 1 : 0;
  a.dt = p->dt;
  a.a_diag = 1.0 + p->q_e / p->De;
  a.q = p->q_e;
  a.s_h = p->s_h;
  a.inv_De = 1.0 / p->De;
  a.tau_scale = p->tau_scale;
  a.eta_e = p->eta_e;
  a.fa = 1.5;
  a.fb = -0.5;
  a.eta = p->eta;
  a.s_ec = p->s_ec;
  if constexpr (BDF2) a.a_diag = p->a_diag;
  const int64_t blocks = (p->npoints * L + kFusedBlock - 1) / kFusedBlock;
  const int per_lane = (p->field_terms + L - 1) / L;
  // the field table goes to LDS when it is small (64 terms: 9 KB in 3-D); with the largest
  // rotated set (64 terms a lane, 128 KB) the block holds at most 160 KB, the CU's whole LDS
  const size_t tab = sizeof(double2) * (((size_t)p->field_terms * (D + 4 + D * D + kTabPad) + 1) / 2);
  const bool lf = tab <= kTabLdsMax;
  const size_t lds = (lf ? tab : 0) +
                     ((!p->field_steady && per_lane <= kRotTerms) ? sizeof(double2) * per_lane * kFusedBlock : 0);
  const void* fn;
  if constexpr (BDF2)
    fn = lf ? reinterpret_cast<const void*>(&fused_bdf2_kernel<D, MT, M, L, true>)
            : reinterpret_cast<const void*>(&fused_bdf2_kernel<D, MT, M, L, false>);
  else
    fn = lf ? reinterpret_cast<const void*>(&fused_exp_kernel<D, MT, M, L, true>)
            : reinterpret_cast<const void*>(&fused_exp_kernel<D, MT, M, L, false>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const dim3 gr((unsigned)blocks), bl(kFusedBlock);
  if constexpr (BDF2) {
    if (lf) hipLaunchKernelGGL((fused_bdf2_kernel<D, MT, M, L, true>), gr, bl, lds, p->stream, a);
    else hipLaunchKernelGGL((fused_bdf2_kernel<D, MT, M, L, false>), gr, bl, lds, p->stream, a);
  } else {
    if (lf) hipLaunchKernelGGL((fused_exp_kernel<D, MT, M, L, true>), gr, bl, lds, p->stream, a);
    else hipLaunchKernelGGL((fused_exp_kernel<D, MT, M, L, false>), gr, bl, lds, p->stream, a);
  }
  return hipGetLastError();
}

}  // namespace

bool fused_supported(const tfs_plan_s* p) {
  if (p->m != 16 && p->m != 32) return false;
  return p->d == 2 || p->precision == TFS_FP32_MODES;
}

hipError_t launch_fused(const tfs_plan_s* p, int64_t n0, int64_t nsteps, double* X, void* Y, double* tau) {
  if (p->npoints == 0 || nsteps == 0) return hipSuccess;
  const bool f32 = p->precision == TFS_FP32_MODES;
  // the exponential scheme: two lanes per point, each with half of the one mode level and of
  // the field's terms; BDF2 (two levels): four lanes per point
  if (p->scheme == TFS_SCHEME_BDF2) {
    if (p->d == 2) {
      if (f32) return p->m == 16 ? fused_go<2, float, 16, 4, true>(p, n0, nsteps, X, Y, tau)
                                 : fused_go<2, float, 32, 4, true>(p, n0, nsteps, X, Y, tau);
      return p->m == 16 ? fused_go<2, double, 16, 4, true>(p, n0, nsteps, X, Y, tau)
                        : fused_go<2, double, 32, 4, true>(p, n0, nsteps, X, Y, tau);
    }
    return p->m == 16 ? fused_go<3, float, 16, 4, true>(p, n0, nsteps, X, Y, tau)
                      : fused_go<3, float, 32, 4, true>(p, n0, nsteps, X, Y, tau);
  }
  if (p->d == 2) {
    if (f32) return p->m == 16 ? fused_go<2, float, 16, 2, false>(p, n0, nsteps, X, Y, tau)
                               : fused_go<2, float, 32, 2, false>(p, n0, nsteps, X, Y, tau);
    return p->m == 16 ? fused_go<2, double, 16, 2, false>(p, n0, nsteps, X, Y, tau)
                      : fused_go<2, double, 32, 2, false>(p, n0, nsteps, X, Y, tau);
  }
  return p->m == 16 ? fused_go<3, float, 16, 2, false>(p, n0, nsteps, X, Y, tau)
                    : fused_go<3, float, 32, 2, false>(p, n0, nsteps, X, Y, tau);
}

}  // namespace tfs

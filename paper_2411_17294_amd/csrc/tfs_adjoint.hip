// Adjoint (reverse-mode) kernels of the time-fractional extra-stress update (gfx950).
//
// The forward BDF2 step is linear in the state, so its transpose runs backwards in time
// with the same streaming structure.  The mode history h^_k = 2 Y_k^n - Y_k^{n-1}/2 enters
// Y_k^{n+1} = d_k h^_k + d_k c_k P and G = sum_k eta_k h^_k + s P; its adjoint
//     H_k^(n) = dL/dh^_k(step n) = d_k Ybar_k^{n+1} + eta_k Gbar^(n),
//     Ybar_k^{j} = 2 H_k^(j) - H_k^(j+1)/2,
// is itself a two-level recurrence: each backward step reads H^(n+1), H^(n+2) and writes
// H^(n) into the slot of H^(n+2).  The forward modes of levels n, n-1 are read only for
// the gradients of the per-mode coefficients (d_k, d_k c_k, eta_k).
//
// Per point the local part is reversed by hand: tau = q (eta X^{n+1} - G), the pivoted solve
// M X^{n+1} = R with M = a I - eta K(kappa~) (adjoint: M^T Rbar = Xbar), R = P - A(G) +
// zeta S, A(G) = K(kappa~) G - G/De.  Gradients with respect to kappa~ use, for a packed
// adjoint v and symmetric Z, v . packed(kappa Z + Z kappa^T) = 2 <V Z, kappa> with V the
// symmetric matrix holding v on the diagonal and v/2 off it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "tfs_device.h"
#include "tfs_internal.h"

namespace tfs {
namespace {
using namespace dev;

// K(kappa) as an explicit packed c x c matrix (column t = K applied to the t-th unit tensor).
template <int D>
__device__ __forceinline__ void build_K(const double (&k)[D * D], double (&Km)[Sym<D>::C][Sym<D>::C]) {
  build_M<D>(k, 0.0, -1.0, Km);
}

// u = K(kappa)^T v on packed tensors: u . z = v . packed(kappa Z + Z kappa^T) for every
// symmetric Z.  With V the symmetric matrix of packed v (v/2 off the diagonal) that inner
// product is <kappa^T V + V kappa, Z>, so u is that matrix packed with its off-diagonal
// entries counted twice.
template <int D>
__device__ __forceinline__ void apply_KT(const double (&k)[D * D], const double (&v)[Sym<D>::C],
                                         double (&u)[Sym<D>::C]) {
  constexpr int C = Sym<D>::C;
  double Vm[D][D];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    const int i = Sym<D>::i(s), j = Sym<D>::j(s);
    const double hv = (i == j) ? v[s] : 0.5 * v[s];
    Vm[i][j] = hv; Vm[j][i] = hv;
  }
#pragma unroll
  for (int s = 0; s < C; ++s) {
    const int i = Sym<D>::i(s), j = Sym<D>::j(s);
    double acc = 0.0;
#pragma unroll
    for (int l = 0; l < D; ++l) acc += k[l * D + i] * Vm[l][j] + Vm[i][l] * k[l * D + j];
    u[s] = (i == j) ? acc : 2.0 * acc;
  }
}

// kb += f * 2 V Z, V the symmetric matrix of packed v (v/2 off the diagonal), Z symmetric packed.
template <int D>
__device__ __forceinline__ void kgrad_VZ(double (&kb)[D * D], double f, const double (&v)[Sym<D>::C],
                                         const double (&z)[Sym<D>::C]) {
  constexpr int C = Sym<D>::C;
  double Vm[D][D], Zm[D][D];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    const int i = Sym<D>::i(s), j = Sym<D>::j(s);
    const double hv = (i == j) ? v[s] : 0.5 * v[s];
    Vm[i][j] = hv; Vm[j][i] = hv;
    Zm[i][j] = z[s]; Zm[j][i] = z[s];
  }
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int j = 0; j < D; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int l = 0; l < D; ++l) acc += Vm[i][l] * Zm[l][j];
      kb[i * D + j] += 2.0 * f * acc;
    }
}

// kb += f * 2 V  (gradient of v . packed(kappa + kappa^T)).
template <int D>
__device__ __forceinline__ void kgrad_V(double (&kb)[D * D], double f, const double (&v)[Sym<D>::C]) {
#pragma unroll
  for (int s = 0; s < Sym<D>::C; ++s) {
    const int i = Sym<D>::i(s), j = Sym<D>::j(s);
    if (i == j) {
      kb[i * D + i] += 2.0 * f * v[s];
    } else {
      kb[i * D + j] += f * v[s];
      kb[j * D + i] += f * v[s];
    }
  }
}

template <int C>
__device__ __forceinline__ double dot(const double (&a)[C], const double (&b)[C]) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < C; ++i) s += a[i] * b[i];
  return s;
}

// Solve M^T x = r (r becomes x) for a packed c x c M given row-major.
template <int N>
__device__ __forceinline__ void solve_transposed(const double (&M)[N][N], double (&r)[N]) {
  double Mt[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) Mt[i][j] = M[j][i];
  solve_pivot<N>(Mt, r);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// v moved across lanes by the DPP pattern CTRL (a permutation inside each row of 16 lanes).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ double lane_value(double v, int l) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Sum over the 64 lanes of a wave (every lane active), the same on every lane and in a
// fixed order: butterflies inside each row of 16 lanes (DPP: swap neighbours, swap pairs,
// rotate by 4, rotate by 8), then the four row sums in row order.
__device__ __forceinline__ double wave_total(double v) {
  v += dpp_mov<0xB1>(v);    // quad_perm(1,0,3,2)
  v += dpp_mov<0x4E>(v);    // quad_perm(2,3,0,1)
  v += dpp_mov<0x124>(v);   // row_ror:4
  v += dpp_mov<0x128>(v);   // row_ror:8
  return ((lane_value(v, 0) + lane_value(v, 16)) + lane_value(v, 32)) + lane_value(v, 48);
}

// Block partial: the per-mode sums (3 rows of m, accumulated per wave in LDS) and the
// per-lane scalar sums, folded over the block in a fixed order and written to part[block].
__device__ inline void write_block_partial(double* __restrict__ part, int m, const double* smode,
                                           const double (&sc)[kNumAdjScalars]) {
  __shared__ double shs[kBlock / 64][kNumAdjScalars];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  double red[kNumAdjScalars];
#pragma unroll
  for (int i = 0; i < kNumAdjScalars; ++i) red[i] = wave_sum(sc[i]);
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < kNumAdjScalars; ++i) shs[wave][i] = red[i];
  __syncthreads();
  const int np = 3 * m + kNumAdjScalars;
  double* o = part + (size_t)blockIdx.x * np;
  for (int j = threadIdx.x; j < 3 * m; j += kBlock) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += smode[w * 3 * m + j];
    o[j] = s;
  }
  if (threadIdx.x < kNumAdjScalars) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += shs[w][threadIdx.x];
    o[3 * m + threadIdx.x] = s;
  }
}

// kbar field += f * kbar of the wave's points (kbar may be null: nothing to do).  Every
// load of the field is issued before any of its stores, so the read-modify-write costs
// one memory latency, not one per component.
template <int D, int V, bool FULL>
__device__ __forceinline__ void add_kbar(double* kb, double f, int64_t st, const WaveAddr& w, int nv,
                                         const double (&kbar)[D * D][V]) {
  if (!kb) return;
  double x[D * D][V];
#pragma unroll
  for (int t = 0; t < D * D; ++t) load_v<FULL, double, V>(at(kb + t * st + w.pw, w.ox), nv, x[t]);
#pragma unroll
  for (int t = 0; t < D * D; ++t)
#pragma unroll
    for (int v = 0; v < V; ++v) x[t][v] += f * kbar[t][v];
#pragma unroll
  for (int t = 0; t < D * D; ++t) store_v<FULL, double, V>(at(kb + t * st + w.pw, w.ox), nv, x[t]);
}

// Spatial form (tfs_plan_set_spatial): each point's extra relaxation rate and whether it is
// the one point that carries the mass-mode source.
struct AdjSpatial {
  const double* rate;   // [stride] or null
  int64_t src;          // the source point, or -1 (every point)
};

// rate and source weight (1 or 0) of the points p0 .. p0 + V - 1 at base + byte offset
template <bool FULL, int V>
__device__ __forceinline__ void adj_spatial(const AdjSpatial& sp, const double* rate_base, int64_t p0, int nv,
                                            double (&rate)[V], double (&srcw)[V]) {
  if (sp.rate) {
    load_v<FULL, double, V>(rate_base, nv, rate);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) rate[v] = 0.0;
  }
#pragma unroll
  for (int v = 0; v < V; ++v) srcw[v] = (sp.src < 0 || p0 + v == sp.src) ? 1.0 : 0.0;
}

// ------------------------------------------------------------------ BDF2 step adjoint
template <typename MT, typename KT>
struct AdjArgs {
  const KT* ka;          // the plan's kappa precision
  const KT* kb;          // null: kappa~ = kappa_a
  const double* Xn;      // forward X^n
  const double* Xm;      // forward X^{n-1}
  const double* Xmm;     // forward X^{n-2} (shifted mode form; null: zero)
  const double* Xp;      // forward X^{n+1}
  const MT* Yn;          // forward Y^n (tiled; Z^n in the shifted form)
  const MT* Ym;          // forward Y^{n-1}
  double* Xb_new;        // adjoint slot (n+1)%L: in Xbar^{n+1}; out partial Xbar^{n-1} (L = 2) or
                         // the part of Xbar^{n-2} from this step (L = 3; at n = 1 the part of the
                         // zero level X^{-1}, which nothing reads)
  double* Xb_cur;        // adjoint slot n%L: in partial Xbar^n, out complete Xbar^n
  double* Xb_old;        // L = 3: slot (n-1)%3, in and out partial Xbar^{n-1}
  const MT* H1;          // H^(n+1) slot (n+1)%2
  MT* H2;                // H^(n+2) in, H^(n) out: slot n%2
  const double* taubar;  // [c][stride] or null
  double* kba;           // kappa_a adjoint (+=) or null
  double* kbb;           // kappa_b adjoint (+=) or null
  int kb_same;           // kba == kbb
  const double* coef;
  double* part;          // block partials: this launch writes part[part0 + block]
  int64_t p_begin;       // first point of this launch
  int64_t ngroups;       // groups of V points from p_begin
  int64_t stride, tile;
  int m, part0;
  Bdf2Scalars s;
  AdjSpatial sp;
};

// Modes of the BDF2 adjoint's four streams loaded ahead of the one being updated (0 or 1;
// measured at 3-D, m = 48: the prefetch holds more registers than it hides latency).
#ifndef TFS_ADJ_AHEAD
#define TFS_ADJ_AHEAD 0
#endif
constexpr int kAdjAhead = TFS_ADJ_AHEAD;

// Per-lane values kept in LDS across the mode stream (they are needed again after it):
// Rbar (c values) and the kappa~ adjoint of the local part (d*d values), per point.
template <int D>
struct AdjSlots {
  static constexpr int N = Sym<D>::C + D * D;
};

// ZF: the shifted mode form (Z_k^j = Y_k^j - beta_k X^{j-1}).  Its history reads back as
// h^_k = 2 Z_k^n - Z_k^{n-1}/2 + beta_k B, B = 2 X^{n-1} - X^{n-2}/2, and its new level is
// Z_k^{n+1} = d_k h^_k + d_k c_k P - beta_k X^n; so with H_k = dL/dh^_k (the same recurrence),
// Bbar = sum_k beta_k H_k reaches X^{n-1} (x 2) and X^{n-2} (x -1/2), and X^n gets
// -sum_k beta_k Zbar_k^{n+1}.  beta_k is a change of representation, not a coefficient of
// the scheme: it has no gradient.
template <int D, typename MT, typename KT, int V, bool FULL, bool SP, bool ZF = false>
__device__ __forceinline__ void adj_group(const AdjArgs<MT, KT>& a, const WaveAddr& w, int nv, double* smode,
                                          double* slot, double (&sc)[kNumAdjScalars]) {
  constexpr int C = Sym<D>::C;
  constexpr int CZ = ZF ? C : 1;
  constexpr int NS = AdjSlots<D>::N;
  const int64_t st = a.stride;
  const int m = a.m;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  auto lds = [&](int v, int j) -> double& { return slot[(v * NS + j) * kBlock + threadIdx.x]; };
  const double q = a.s.tau_scale, eta = a.s.eta;

  // ---- local part, point by point: Rbar = M^{-T} Xbar and everything that needs kappa~
  double Gb[C][V], Pb[C][V];
  {
    double kt[D * D][V], Xp[C][V], Xbn[C][V], tb[C][V];
    const uint32_t kx = field_off<KT>(w.ox);
#pragma unroll
    for (int t = 0; t < D * D; ++t) {
      KT x[V];
      load_v<FULL, KT, V>(at(a.ka + t * st + w.pw, kx), nv, x);
      if (a.kb) {
        KT y[V];
        load_v<FULL, KT, V>(at(a.kb + t * st + w.pw, kx), nv, y);
#pragma unroll
        for (int v = 0; v < V; ++v) kt[t][v] = 2.0 * (double)x[v] - (double)y[v];
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) kt[t][v] = (double)x[v];
      }
    }
#pragma unroll
    for (int s = 0; s < C; ++s) {
      load_v<FULL, double, V>(at(a.Xp + s * st + w.pw, w.ox), nv, Xp[s]);
      load_v<FULL, double, V>(at(a.Xb_new + s * st + w.pw, w.ox), nv, Xbn[s]);
      if (a.taubar) load_v<FULL, double, V>(at(a.taubar + s * st + w.pw, w.ox), nv, tb[s]);
      else
#pragma unroll
        for (int v = 0; v < V; ++v) tb[s][v] = 0.0;
    }
    double rate[V], srcw[V];
    if constexpr (SP) adj_spatial<FULL, V>(a.sp, at(a.sp.rate + w.pw, w.ox), w.pw + (int64_t)(w.ox / 8), nv, rate, srcw);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      double k[D * D], xp[C], rb[C], tv[C], S[C];
      // spatial form: 1/De + rate, the diagonal a + eta rate, the source weight
      const double idv = SP ? a.s.inv_De + rate[v] : a.s.inv_De;
      const double adg = SP ? a.s.a_diag + eta * rate[v] : a.s.a_diag;
      const double zw = SP ? a.s.zeta * srcw[v] : a.s.zeta;
#pragma unroll
      for (int t = 0; t < D * D; ++t) k[t] = kt[t][v];
#pragma unroll
      for (int s = 0; s < C; ++s) {
        xp[s] = Xp[s][v];
        tv[s] = tb[s][v];
        rb[s] = Xbn[s][v] + q * eta * tv[s];        // tau = q (eta X+ - G)
        const int i = Sym<D>::i(s), j = Sym<D>::j(s);
        S[s] = k[i * D + j] + k[j * D + i];
      }
      sc[1] += q * dot<C>(tv, xp);                  // d tau / d eta (X+ part)
      sc[4] += eta * dot<C>(tv, xp);                // d tau / d q (X+ part; the G part follows the modes)
      {
        double M[C][C];
        build_M<D>(k, adg, eta, M);
        solve_transposed<C>(M, rb);                 // Rbar = M^{-T} Xbar
      }
      double Kx[C];
      apply_K<D>(k, xp, Kx);
      const double ra = -dot<C>(rb, xp);
      sc[0] += ra;                                  // a
      sc[1] += dot<C>(rb, Kx);                      // eta (matrix)
      if constexpr (SP) {
        sc[5] += srcw[v] * dot<C>(rb, S);           // zeta (the source point only)
        sc[6] += rate[v] * ra;                      // eta through a + eta rate
        sc[7] += rate[v] * eta * ra;                // rate through a + eta rate
      } else {
        sc[5] += dot<C>(rb, S);                     // zeta
      }
      double kb_[D * D];
#pragma unroll
      for (int t = 0; t < D * D; ++t) kb_[t] = 0.0;
      kgrad_VZ<D>(kb_, eta, rb, xp);                // M = a I - eta K(kappa)
      kgrad_V<D>(kb_, zw, rb);                      // R = ... + zeta S
      // A(G) = K G - G/De with AGbar = -Rbar:  Gbar = K^T AGbar - AGbar/De - q taubar
      double u[C];
      apply_KT<D>(k, rb, u);
#pragma unroll
      for (int t = 0; t < C; ++t) {
        Gb[t][v] = -u[t] + idv * rb[t] - q * tv[t];
        Pb[t][v] = rb[t] + a.s.s_ec * Gb[t][v];     // P enters R directly and through G = G^ + s P
      }
#pragma unroll
      for (int s = 0; s < C; ++s) lds(v, s) = rb[s];
#pragma unroll
      for (int t = 0; t < D * D; ++t) lds(v, C + t) = kb_[t];
    }
  }

  double P[C][V], B[CZ][V];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    double xn[V], xm[V];
    load_v<FULL, double, V>(at(a.Xn + s * st + w.pw, w.ox), nv, xn);
    load_v<FULL, double, V>(at(a.Xm + s * st + w.pw, w.ox), nv, xm);
#pragma unroll
    for (int v = 0; v < V; ++v) P[s][v] = 2.0 * xn[v] - 0.5 * xm[v];
    if constexpr (ZF) {
      double xmm[V];
      if (a.Xmm) {
        load_v<FULL, double, V>(at(a.Xmm + s * st + w.pw, w.ox), nv, xmm);
      } else {
#pragma unroll
        for (int v = 0; v < V; ++v) xmm[v] = 0.0;
      }
#pragma unroll
      for (int v = 0; v < V; ++v) B[s][v] = 2.0 * xm[v] - 0.5 * xmm[v];
    }
  }
  {
    double g = 0.0;
#pragma unroll
    for (int s = 0; s < C; ++s)
#pragma unroll
      for (int v = 0; v < V; ++v) g += Gb[s][v] * P[s][v];
    sc[2] += g;                                     // G = G^ + s P
  }

  // ---- transposed mode recurrence, streaming
  const int64_t T = a.tile;
  const MT* h1p = a.H1 + w.tw;
  MT* h2p = a.H2 + w.tw;
  const MT* ynp = a.Yn + w.tw;
  const MT* ymp = a.Ym + w.tw;
  double Gh[C][V], Bb[CZ][V], Zx[CZ][V];   // Bbar and -sum_k beta_k Zbar_k^{n+1} (shifted form)
#pragma unroll
  for (int s = 0; s < C; ++s)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      Gh[s][v] = 0.0;
      if constexpr (ZF) {
        Bb[s][v] = 0.0;
        Zx[s][v] = 0.0;
      }
    }
  // the four streams of mode k + 1 are loaded before mode k's arithmetic, reductions and
  // store, so a wave keeps its next loads in flight while it works (H^(n+2) of mode k + 1 is
  // read before H^(n) of mode k is written into the same slot: different addresses)
  MT c1[C][V], c2[C][V], cn[C][V], cm[C][V];
  auto load_mode = [&](int k, MT (&x1)[C][V], MT (&x2)[C][V], MT (&xn)[C][V], MT (&xm)[C][V]) {
    const int64_t o = (int64_t)k * C * T;
    const uint32_t om = opaque(w.om);
    const MT* b1 = opaque_ptr(h1p + o);
    const MT* b2 = opaque_ptr(h2p + o);
    const MT* bn = opaque_ptr(ynp + o);
    const MT* bm = opaque_ptr(ymp + o);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      load_v<FULL, MT, V, true>(at(b1 + s * T, om), nv, x1[s]);
      load_v<FULL, MT, V, true>(at(b2 + s * T, om), nv, x2[s]);
      load_v<FULL, MT, V, true>(at(bn + s * T, om), nv, xn[s]);
      load_v<FULL, MT, V, true>(at(bm + s * T, om), nv, xm[s]);
    }
  };
  if constexpr (kAdjAhead) load_mode(0, c1, c2, cn, cm);
  for (int k = 0; k < m; ++k) {
    const double dk = load_uniform(a.coef + kRowD * m + k);
    const double ek = load_uniform(a.coef + kRowDC * m + k);
    const double hk = load_uniform(a.coef + kRowEta * m + k);
    const double bk = ZF ? load_uniform(a.coef + kRowBeta * m + k) : 0.0;
    MT n1[C][V], n2[C][V], nn[C][V], nm[C][V];
    if constexpr (kAdjAhead) {
      if (k + 1 < m) load_mode(k + 1, n1, n2, nn, nm);
    } else {
      load_mode(k, c1, c2, cn, cm);
    }
    const uint32_t om = opaque(w.om);
    MT* b2 = opaque_ptr(h2p + (int64_t)k * C * T);
    double ad = 0.0, ae = 0.0, ah = 0.0;
#pragma unroll
    for (int s = 0; s < C; ++s) {
      MT hv[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double yb = 2.0 * (double)c1[s][v] - 0.5 * (double)c2[s][v];
        double hh = 2.0 * (double)cn[s][v] - 0.5 * (double)cm[s][v];
        if constexpr (ZF) hh += bk * B[s][v];
        Gh[s][v] += hk * hh;
        const double hn = dk * yb + hk * Gb[s][v];
        hv[v] = (MT)hn;
        if constexpr (ZF) {
          Bb[s][v] += bk * hn;
          Zx[s][v] -= bk * yb;
        }
        Pb[s][v] += ek * yb;
        ad += yb * hh;
        ae += yb * P[s][v];
        ah += Gb[s][v] * hh;
      }
      store_v<FULL, MT, V, true>(at(b2 + s * T, om), nv, hv);
    }
    ad = wave_total(ad);
    ae = wave_total(ae);
    ah = wave_total(ah);
    if (lane == 0) {
      smode[wave * 3 * m + k] += ad;
      smode[wave * 3 * m + m + k] += ae;
      smode[wave * 3 * m + 2 * m + k] += ah;
    }
    if (kAdjAhead && k + 1 < m) {
#pragma unroll
      for (int s = 0; s < C; ++s)
#pragma unroll
        for (int v = 0; v < V; ++v) {
          c1[s][v] = n1[s][v];
          c2[s][v] = n2[s][v];
          cn[s][v] = nn[s][v];
          cm[s][v] = nm[s][v];
        }
    }
  }

  // ---- terms that need G = G^ + s P, the X adjoints and the kappa adjoints
  double kbar[D * D][V];
  {
    double tb[C][V];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      if (a.taubar) load_v<FULL, double, V>(at(a.taubar + s * st + w.pw, w.ox), nv, tb[s]);
      else
#pragma unroll
        for (int v = 0; v < V; ++v) tb[s][v] = 0.0;
    }
    double rate[V], srcw[V];
    if constexpr (SP) adj_spatial<FULL, V>(a.sp, at(a.sp.rate + w.pw, w.ox), w.pw + (int64_t)(w.ox / 8), nv, rate, srcw);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      double G[C], rb[C], tv[C], kb_[D * D];
#pragma unroll
      for (int s = 0; s < C; ++s) {
        G[s] = Gh[s][v] + a.s.s_ec * P[s][v];
        rb[s] = lds(v, s);
        tv[s] = tb[s][v];
      }
#pragma unroll
      for (int t = 0; t < D * D; ++t) kb_[t] = lds(v, C + t);
      const double rg = dot<C>(rb, G);
      sc[3] += rg;                                  // 1/De (AGbar = -Rbar)
      if constexpr (SP) sc[7] += rate[v] * rg;      // rate through 1/De + rate
      sc[4] += -dot<C>(tv, G);                      // q (G part)
      kgrad_VZ<D>(kb_, -1.0, rb, G);                // A(G) = K(kappa) G - G/De
#pragma unroll
      for (int t = 0; t < D * D; ++t) kbar[t][v] = kb_[t];
    }
  }
#pragma unroll
  for (int s = 0; s < C; ++s) {
    double xc[V], xw[V];
    load_v<FULL, double, V>(at(a.Xb_cur + s * st + w.pw, w.ox), nv, xc);
    if constexpr (ZF) {
      // three slots: Xbar^n complete, Xbar^{n-1} accumulated, Xbar^{n-2} started
      double xo[V];
      load_v<FULL, double, V>(at(a.Xb_old + s * st + w.pw, w.ox), nv, xo);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        xc[v] += 2.0 * Pb[s][v] + Zx[s][v];         // P = 2 X^n - X^{n-1}/2; Z^{n+1} = ... - beta X^n
        xo[v] += -0.5 * Pb[s][v] + 2.0 * Bb[s][v];  // B = 2 X^{n-1} - X^{n-2}/2
        xw[v] = -0.5 * Bb[s][v];
      }
      store_v<FULL, double, V>(at(a.Xb_old + s * st + w.pw, w.ox), nv, xo);
      store_v<FULL, double, V>(at(a.Xb_new + s * st + w.pw, w.ox), nv, xw);
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        xc[v] += 2.0 * Pb[s][v];                      // P = 2 X^n - X^{n-1}/2
        xw[v] = -0.5 * Pb[s][v];
      }
      store_v<FULL, double, V>(at(a.Xb_new + s * st + w.pw, w.ox), nv, xw);
    }
    store_v<FULL, double, V>(at(a.Xb_cur + s * st + w.pw, w.ox), nv, xc);
  }
  // kappa adjoints: kappa~ = 2 kappa_a - kappa_b, or kappa_a
  double fa = 1.0, fb = 0.0;
  if (a.kb && !a.kb_same) { fa = 2.0; fb = -1.0; }
  add_kbar<D, V, FULL>(a.kba, fa, st, w, nv, kbar);
  if (a.kbb && fb != 0.0) add_kbar<D, V, FULL>(a.kbb, fb, st, w, nv, kbar);
}

// FULL: whole waves of V-point groups (ngroups a multiple of 64).  !FULL (V = 1): the
// points after the last whole wave; lanes past the end run an empty group, since the wave
// reductions need all 64 lanes.
// Optional lower bound on the waves per SIMD the BDF2 adjoint is compiled for (0: the
// compiler's choice); it caps the registers a lane may hold.
#ifndef TFS_ADJ_WAVES
#define TFS_ADJ_WAVES 0
#endif
#if TFS_ADJ_WAVES > 0
#define TFS_ADJ_ATTR __attribute__((amdgpu_waves_per_eu(TFS_ADJ_WAVES)))
#else
#define TFS_ADJ_ATTR
#endif

template <int D, typename MT, typename KT, int V, bool FULL, bool SP, bool ZF>
__global__ __launch_bounds__(kBlock) TFS_ADJ_ATTR void adj_kernel(const AdjArgs<MT, KT> a) {
  constexpr int C = Sym<D>::C;
  extern __shared__ double smem[];    // [kBlock/64][3][m] mode sums, then the lane slots
  double* smode = smem;
  double* slot = smem + (kBlock / 64) * 3 * a.m;
  for (int j = threadIdx.x; j < (kBlock / 64) * 3 * a.m; j += kBlock) smode[j] = 0.0;
  __syncthreads();
  double sc[kNumAdjScalars];
#pragma unroll
  for (int i = 0; i < kNumAdjScalars; ++i) sc[i] = 0.0;
  const int lane = threadIdx.x % 64;
  const int64_t nwaves = (a.ngroups + 63) / 64;
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / 64);
  for (int64_t wv = wave_uniform((int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64); wv < nwaves;
       wv += wstride) {
    const WaveAddr w = wave_addr<MT, C, V>(a.p_begin + wv * 64 * V, lane, a.tile, a.m);
    const int nv = (FULL || wv * 64 + lane < a.ngroups) ? V : 0;
    adj_group<D, MT, KT, V, FULL, SP, ZF>(a, w, nv, smode, slot, sc);
  }
  __syncthreads();
  write_block_partial(a.part + (size_t)a.part0 * (3 * a.m + kNumAdjScalars), a.m, smode, sc);
}

// ------------------------------------------------------------------ exponential-mode step adjoint
// Reverse of the TFS_SCHEME_EXP step (the forward is in the step kernels' source):
//   Y_k^{n+1} = e_k Y_k^n + f_k X^n,  H = sum_k om_k Y_k^n + s_h X^n,  G = sum_k l_k Y_k^{n+1},
//   M X^{n+1} = X^n - A(H) + zeta S (M = a I - q K),  tau = ts (eta_e X^{n+1} - G).
// With Gbar = -ts taubar, Rbar = M^{-T}(Xbar^{n+1} + ts eta_e taubar), Hbar = -K^T Rbar + Rbar/De:
//   Yhat_k = Ybar_k^{n+1} + l_k Gbar,   Ybar_k^n = e_k Yhat_k + om_k Hbar   (one level, in place)
//   Xbar^n = Rbar + s_h Hbar + sum_k f_k Yhat_k   (at n = 0 also - sum_k q_k Ybar_k^0)
// and per mode dL/dw_k, dL/dlambda_k through e_k, f_k, om_k, l_k (and q_k at n = 0).
template <typename MT, typename KT>
struct ExpAdjArgs {
  const KT* ka;          // the plan's kappa precision
  const KT* kb;          // null: kappa~ = kappa_a
  const double* Xn;      // forward X^n
  const double* Xp;      // forward X^{n+1}
  const MT* Yn;          // forward Y^n (one level, tiled); not read at n = 0
  const double* Xb_in;   // Xbar^{n+1} (ring slot (n+1)%2)
  double* Xb_out;        // Xbar^n (ring slot n%2), overwritten
  MT* H;                 // Ybar^{n+1} in, Ybar^n out (one level); not written at n = 0
  const double* taubar;  // [c][stride] or null
  double* kba;           // kappa_a adjoint (+=) or null
  double* kbb;           // kappa_b adjoint (+=) or null
  int kb_same;
  const double* coef;
  double* part;
  int64_t p_begin, ngroups;
  int64_t stride, tile;
  int m, part0;
  ExpScalars s;
  double dt;
  AdjSpatial sp;
};

// TAU: this step's stress is in the loss (taubar given: the last step of a misfit).  Without
// it Gbar = 0, and neither G nor the recomputed Y^{n+1} is needed.
#ifndef TFS_EXP_ADJ_AHEAD
#define TFS_EXP_ADJ_AHEAD 1
#endif
// modes whose forward and adjoint loads are in flight ahead of the one being updated
constexpr int kExpAdjAhead = TFS_EXP_ADJ_AHEAD;

// SP: the spatial form (1/De + rate per point, a + q rate on the diagonal, the mass-mode
// source at the source point only); sc[7] collects sum rate dL/da (a part of dL/dq) and sc[8]
// sum rate dL/drate.
template <int D, typename MT, typename KT, int V, bool FULL, bool TAU, bool SP>
__device__ __forceinline__ void exp_adj_group(const ExpAdjArgs<MT, KT>& a, const WaveAddr& w, int nv, double* smode,
                                              double* slot, double (&sc)[kNumAdjScalars]) {
  constexpr int C = Sym<D>::C;
  const int64_t st = a.stride;
  const int m = a.m;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const bool first = a.s.first != 0;
  auto lds = [&](int v, int j) -> double& { return slot[(v * C + j) * kBlock + threadIdx.x]; };
  const double ts = a.s.tau_scale, eta_e = a.s.eta_e, q = a.s.q;

  // ---- local part, point by point
  double Gb[TAU ? C : 1][V], Hb[C][V], Xc[C][V], Xacc[C][V];
  double rate[V], srcw[V];
  if constexpr (SP) adj_spatial<FULL, V>(a.sp, at(a.sp.rate + w.pw, w.ox), w.pw + (int64_t)(w.ox / 8), nv, rate, srcw);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const double idv = SP ? a.s.inv_De + rate[v] : a.s.inv_De;
    const double adg = SP ? a.s.a_diag + q * rate[v] : a.s.a_diag;
    const uint32_t ox = w.ox + v * 8;
    const int nv1 = v < nv ? 1 : 0;
    double k[D * D], xp[C], rb[C], tv[C], S[C];
#pragma unroll
    for (int t = 0; t < D * D; ++t) {
      KT x[1];
      load_v<FULL, KT, 1>(at(a.ka + t * st + w.pw, field_off<KT>(ox)), nv1, x);
      k[t] = (double)x[0];
    }
    if (a.kb) {
      double kb[D * D];
#pragma unroll
      for (int t = 0; t < D * D; ++t) {
        KT x[1];
        load_v<FULL, KT, 1>(at(a.kb + t * st + w.pw, field_off<KT>(ox)), nv1, x);
        kb[t] = (double)x[0];
      }
#pragma unroll
      for (int t = 0; t < D * D; ++t) k[t] = a.s.fa * k[t] + a.s.fb * kb[t];
    }
#pragma unroll
    for (int s = 0; s < C; ++s) {
      double x[1];
      load_v<FULL, double, 1>(at(a.Xp + s * st + w.pw, ox), nv1, x);
      xp[s] = x[0];
      tv[s] = 0.0;
      if constexpr (TAU) {
        load_v<FULL, double, 1>(at(a.taubar + s * st + w.pw, ox), nv1, x);
        tv[s] = x[0];
      }
      load_v<FULL, double, 1>(at(a.Xb_in + s * st + w.pw, ox), nv1, x);
      rb[s] = x[0] + ts * eta_e * tv[s];          // tau = ts (eta_e X+ - G)
      load_v<FULL, double, 1>(at(a.Xn + s * st + w.pw, ox), nv1, x);
      Xc[s][v] = x[0];
      const int i = Sym<D>::i(s), j = Sym<D>::j(s);
      S[s] = k[i * D + j] + k[j * D + i];
    }
    if constexpr (TAU) {
      sc[4] += ts * dot<C>(tv, xp);                // eta_e
      sc[6] += eta_e * dot<C>(tv, xp);             // ts (X+ part; the G part follows the modes)
    }
    {
      double M[C][C];
      build_M<D>(k, adg, q, M);
      solve_transposed<C>(M, rb);                  // Rbar = M^{-T} Xbar
    }
    double Kx[C], u[C];
    apply_K<D>(k, xp, Kx);
    const double ra = -dot<C>(rb, xp);
    sc[0] += ra;                                   // a
    sc[1] += dot<C>(rb, Kx);                       // q (matrix)
    if constexpr (SP) {
      sc[5] += srcw[v] * dot<C>(rb, S);            // zeta (the source point only)
      sc[7] += rate[v] * ra;                       // q through a + q rate
      sc[8] += rate[v] * q * ra;                   // rate through a + q rate
    } else {
      sc[5] += dot<C>(rb, S);                      // zeta
    }
    apply_KT<D>(k, rb, u);
#pragma unroll
    for (int t = 0; t < C; ++t) {
      Hb[t][v] = -u[t] + idv * rb[t];              // R = X^n - K H + H (1/De + rate)
      if constexpr (TAU) Gb[t][v] = -ts * tv[t];
      Xacc[t][v] = rb[t] + a.s.s_h * Hb[t][v];
      lds(v, t) = rb[t];
    }
    double hx = 0.0;
#pragma unroll
    for (int t = 0; t < C; ++t) hx += Hb[t][v] * Xc[t][v];
    sc[2] += hx;                                   // s_h
    // one c x c solve live at a time
    __builtin_amdgcn_sched_barrier(0);
  }

  // ---- mode stream: forward Y^n and the adjoint level, in place
  const int64_t T = a.tile;
  const MT* yp = a.Yn + w.tw;
  MT* hp = a.H + w.tw;
  double Hs[C][V], Gs[TAU ? C : 1][V];
#pragma unroll
  for (int s = 0; s < C; ++s)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      Hs[s][v] = 0.0;
      if constexpr (TAU) Gs[s][v] = 0.0;
    }
  // ring of the next kExpAdjAhead modes' two streams
  MT py[kExpAdjAhead][C][V], ph[kExpAdjAhead][C][V];
#pragma unroll
  for (int j = 0; j < kExpAdjAhead; ++j) {
    const uint32_t om = opaque(w.om);
    const int64_t o = (int64_t)j * C * T;
    const MT* by = opaque_ptr(yp + o);
    const MT* bh = opaque_ptr(hp + o);
#pragma unroll
    for (int s = 0; s < C; ++s) {
#pragma unroll
      for (int v = 0; v < V; ++v) { py[j][s][v] = MT(0); ph[j][s][v] = MT(0); }
      if (j < m) {
        if (!first) load_v<FULL, MT, V, true>(at(by + s * T, om), nv, py[j][s]);
        load_v<FULL, MT, V, true>(at(bh + s * T, om), nv, ph[j][s]);
      }
    }
  }
  for (int k = 0; k < m; ++k) {
    const double ek = load_uniform(a.coef + kRowE * m + k);
    const double fk = load_uniform(a.coef + kRowF * m + k);
    const double lk = load_uniform(a.coef + kRowLdt * m + k);
    const double qk = load_uniform(a.coef + kRowQ * m + k);
    const double ok = load_uniform(a.coef + kRowOneME * m + k);
    const double fw = load_uniform(a.coef + kRowFW * m + k);
    const double fl = load_uniform(a.coef + kRowFL * m + k);
    const double qw = load_uniform(a.coef + kRowQW * m + k);
    const double ql = load_uniform(a.coef + kRowQL * m + k);
    const double edt = ek * a.dt;
    // mode k leaves the ring; mode k + kExpAdjAhead is loaded before this mode's arithmetic
    MT cy[C][V], ch[C][V];
#pragma unroll
    for (int s = 0; s < C; ++s)
#pragma unroll
      for (int v = 0; v < V; ++v) {
        cy[s][v] = py[0][s][v];
        ch[s][v] = ph[0][s][v];
#pragma unroll
        for (int j = 0; j + 1 < kExpAdjAhead; ++j) { py[j][s][v] = py[j + 1][s][v]; ph[j][s][v] = ph[j + 1][s][v]; }
      }
    if (k + kExpAdjAhead < m) {
      const uint32_t om = opaque(w.om);
      const int64_t o = (int64_t)(k + kExpAdjAhead) * C * T;
      const MT* by = opaque_ptr(yp + o);
      const MT* bh = opaque_ptr(hp + o);
#pragma unroll
      for (int s = 0; s < C; ++s) {
        if (!first) load_v<FULL, MT, V, true>(at(by + s * T, om), nv, py[kExpAdjAhead - 1][s]);
        load_v<FULL, MT, V, true>(at(bh + s * T, om), nv, ph[kExpAdjAhead - 1][s]);
      }
    }
    double gw = 0.0, gl = 0.0;
    const uint32_t om = opaque(w.om);
    MT* bo = opaque_ptr(hp + (int64_t)k * C * T);
#pragma unroll
    for (int s = 0; s < C; ++s) {
      MT out[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double x = Xc[s][v];
        const double y = first ? -qk * x : (double)cy[s][v];
        double yh = (double)ch[s][v];                              // Yhat = Ybar^{n+1} + l_k Gbar
        if constexpr (TAU) {
          const double yn1 = (double)(MT)(ek * y + fk * x);        // forward Y^{n+1} as stored
          yh += lk * Gb[s][v];
          Gs[s][v] += lk * yn1;
          gl += a.dt * (Gb[s][v] * yn1);
        }
        const double yb = ek * yh + ok * Hb[s][v];                 // Ybar^n
        Hs[s][v] += ok * y;
        Xacc[s][v] += fk * yh;
        gw += fw * (yh * x);
        gl += edt * ((Hb[s][v] - yh) * y) + fl * (yh * x);
        if (first) {
          Xacc[s][v] -= qk * yb;                                   // Y^0 = -q_k X^0
          gw += qw * (yb * x);
          gl += ql * (yb * x);
        }
        out[v] = (MT)yb;
      }
      if (!first) store_v<FULL, MT, V, true>(at(bo + s * T, om), nv, out);
    }
    gw = wave_total(gw);
    gl = wave_total(gl);
    if (lane == 0) {
      smode[wave * 3 * m + k] += gw;
      smode[wave * 3 * m + m + k] += gl;
    }
  }

#pragma unroll
  for (int s = 0; s < C; ++s) store_v<FULL, double, V>(at(a.Xb_out + s * st + w.pw, w.ox), nv, Xacc[s]);

  // ---- terms that need H and G, and the kappa adjoints
  double kbar[D * D][V];
  {
    double Xp[C][V];
#pragma unroll
    for (int s = 0; s < C; ++s) load_v<FULL, double, V>(at(a.Xp + s * st + w.pw, w.ox), nv, Xp[s]);
    if constexpr (SP) adj_spatial<FULL, V>(a.sp, at(a.sp.rate + w.pw, w.ox), w.pw + (int64_t)(w.ox / 8), nv, rate, srcw);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      double Hv[C], Z[C], rb[C], kb_[D * D];
#pragma unroll
      for (int s = 0; s < C; ++s) {
        Hv[s] = Hs[s][v] + a.s.s_h * Xc[s][v];
        Z[s] = q * Xp[s][v] - Hv[s];               // M X+ = R: -q K X+ in M, -K H in R
        rb[s] = lds(v, s);
      }
      if constexpr (TAU) {
        // taubar = -Gbar / ts
        double gv = 0.0;
#pragma unroll
        for (int s = 0; s < C; ++s) gv += Gb[s][v] * Gs[s][v];
        sc[6] += gv / ts;                          // ts (G part): -taubar . G
      }
      const double rh = dot<C>(rb, Hv);
      sc[3] += rh;                                 // 1/De
      if constexpr (SP) sc[8] += rate[v] * rh;     // rate through 1/De + rate
#pragma unroll
      for (int t = 0; t < D * D; ++t) kb_[t] = 0.0;
      kgrad_VZ<D>(kb_, 1.0, rb, Z);
      kgrad_V<D>(kb_, SP ? a.s.zeta * srcw[v] : a.s.zeta, rb);
#pragma unroll
      for (int t = 0; t < D * D; ++t) kbar[t][v] = kb_[t];
    }
  }
  double fa = 1.0, fb = 0.0;
  if (a.kb && !a.kb_same) { fa = a.s.fa; fb = a.s.fb; }
  else if (a.kb && a.kb_same) { fa = a.s.fa + a.s.fb; fb = 0.0; }
  add_kbar<D, V, FULL>(a.kba, fa, st, w, nv, kbar);
  if (a.kbb && fb != 0.0) add_kbar<D, V, FULL>(a.kbb, fb, st, w, nv, kbar);
}

template <int D, typename MT, typename KT, int V, bool FULL, bool TAU, bool SP>
__global__ __launch_bounds__(kBlock) void exp_adj_kernel(const ExpAdjArgs<MT, KT> a) {
  constexpr int C = Sym<D>::C;
  extern __shared__ double smem[];    // [kBlock/64][3][m] mode sums, then Rbar per lane
  double* smode = smem;
  double* slot = smem + (kBlock / 64) * 3 * a.m;
  for (int j = threadIdx.x; j < (kBlock / 64) * 3 * a.m; j += kBlock) smode[j] = 0.0;
  __syncthreads();
  double sc[kNumAdjScalars];
#pragma unroll
  for (int i = 0; i < kNumAdjScalars; ++i) sc[i] = 0.0;
  const int lane = threadIdx.x % 64;
  const int64_t nwaves = (a.ngroups + 63) / 64;
  const int64_t wstride = (int64_t)gridDim.x * (kBlock / 64);
  for (int64_t wv = wave_uniform((int64_t)blockIdx.x * (kBlock / 64) + threadIdx.x / 64); wv < nwaves;
       wv += wstride) {
    const WaveAddr w = wave_addr<MT, C, V>(a.p_begin + wv * 64 * V, lane, a.tile, a.m);
    const int nv = (FULL || wv * 64 + lane < a.ngroups) ? V : 0;
    exp_adj_group<D, MT, KT, V, FULL, TAU, SP>(a, w, nv, smode, slot, sc);
  }
  __syncthreads();
  write_block_partial(a.part + (size_t)a.part0 * (3 * a.m + kNumAdjScalars), a.m, smode, sc);
}

// ------------------------------------------------------------------ start-up adjoint
template <typename MT, typename KT>
struct StartAdjArgs {
  const KT* ka;          // the plan's kappa precision
  const double* X0;      // forward X^0
  double* Xb0;           // adjoint slot 0: in partial Xbar^0, out complete Xbar^0
  const double* Xb1;     // adjoint slot 1: Xbar^1 from later steps
  const MT* H1;          // H^(1) (slot 1)
  const MT* H2;          // H^(2) (slot 0)
  const double* taubar;
  double* kba;
  const double* coef;
  double* part;
  int64_t npts, stride, tile;
  int m;
  int zform;             // shifted mode form: Z^1 = Y^1 - beta_k X^0
  StartScalars s;
  AdjSpatial sp;
};

template <int D, typename MT, typename KT, int V, bool FULL, bool SP>
__device__ __forceinline__ void start_adj_group(const StartAdjArgs<MT, KT>& a, int64_t p0, int nv, double* smode,
                                                double (&sc)[kNumAdjScalars]) {
  constexpr int C = Sym<D>::C;
  const int64_t st = a.stride;
  const int m = a.m;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  double X0[C][V], X1[C][V], X2[C][V], kt[D * D][V];
#pragma unroll
  for (int s = 0; s < C; ++s) load_v<FULL, double, V>(a.X0 + s * st + p0, nv, X0[s]);
#pragma unroll
  for (int q = 0; q < D * D; ++q) {
    KT x[V];
    load_v<FULL, KT, V>(a.ka + q * st + p0, nv, x);
#pragma unroll
    for (int v = 0; v < V; ++v) kt[q][v] = (double)x[v];
  }
  // spatial form: 1/De + rate per point and the source weight of the mass-mode terms
  double rate[V], srcw[V];
  if constexpr (SP) adj_spatial<FULL, V>(a.sp, a.sp.rate + p0, p0, nv, rate, srcw);
  // forward recomputation of the two stages
#pragma unroll
  for (int v = 0; v < V; ++v) {
    double k[D * D], S[C], r[C], M[C][C], AX[C], x1[C];
    const double idv = SP ? a.s.inv_De + rate[v] : a.s.inv_De;
    const double s1 = SP ? a.s.src1 * srcw[v] : a.s.src1;
    const double s2 = SP ? a.s.sigma2 * srcw[v] : a.s.sigma2;
#pragma unroll
    for (int t = 0; t < D * D; ++t) k[t] = kt[t][v];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const int i = Sym<D>::i(s), j = Sym<D>::j(s);
      S[s] = k[i * D + j] + k[j * D + i];
      r[s] = X0[s][v] + s1 * S[s];
    }
    build_M<D>(k, 1.0 + a.s.hgt * idv, a.s.hgt, M);
    solve_pivot<C>(M, r);
#pragma unroll
    for (int s = 0; s < C; ++s) { x1[s] = r[s]; X1[s][v] = r[s]; }
    apply_K<D>(k, x1, AX);
#pragma unroll
    for (int s = 0; s < C; ++s) r[s] = X0[s][v] + a.s.sigma1 * (AX[s] - idv * x1[s]) + s2 * S[s];
    build_M<D>(k, 1.0 + a.s.hgt * idv, a.s.hgt, M);
    solve_pivot<C>(M, r);
#pragma unroll
    for (int s = 0; s < C; ++s) X2[s][v] = r[s];
  }
  // modes: Ybar^0 = -H^(1)/2, Ybar^1 = 2 H^(1) - H^(2)/2;  Y^0 = -c X^0, Y^1 = u X^(1) + v X^(2)
  double X0b[C][V], X1b[C][V], X2b[C][V];
#pragma unroll
  for (int s = 0; s < C; ++s)
#pragma unroll
    for (int v = 0; v < V; ++v) { X0b[s][v] = 0.0; X1b[s][v] = 0.0; X2b[s][v] = 0.0; }
  const int64_t T = a.tile;
  const int64_t toff = (p0 / T) * (int64_t)m * C * T + (p0 % T);
  const MT* h1p = a.H1 + toff;
  const MT* h2p = a.H2 + toff;
  for (int k = 0; k < m; ++k) {
    const double ck = load_uniform(a.coef + kRowC * m + k);
    const double uk = load_uniform(a.coef + kRowU * m + k);
    const double vk = load_uniform(a.coef + kRowV * m + k);
    const double bk = a.zform ? load_uniform(a.coef + kRowBeta * m + k) : 0.0;
    double ac = 0.0, au = 0.0, av = 0.0;
#pragma unroll
    for (int s = 0; s < C; ++s) {
      MT h1[V], h2[V];
      load_v<FULL, MT, V, true>(h1p + ((int64_t)k * C + s) * T, nv, h1);
      load_v<FULL, MT, V, true>(h2p + ((int64_t)k * C + s) * T, nv, h2);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double y0 = -0.5 * (double)h1[v];
        const double y1 = 2.0 * (double)h1[v] - 0.5 * (double)h2[v];
        X0b[s][v] += -ck * y0 - bk * y1;
        X1b[s][v] += uk * y1;
        X2b[s][v] += vk * y1;
        ac += -y0 * X0[s][v];
        au += y1 * X1[s][v];
        av += y1 * X2[s][v];
      }
    }
    ac = wave_sum(ac);
    au = wave_sum(au);
    av = wave_sum(av);
    if (lane == 0) {
      smode[wave * 3 * m + k] += ac;
      smode[wave * 3 * m + m + k] += au;
      smode[wave * 3 * m + 2 * m + k] += av;
    }
  }
  double Xb1[C][V], tb[C][V], Xb0in[C][V];
#pragma unroll
  for (int s = 0; s < C; ++s) {
    load_v<FULL, double, V>(a.Xb1 + s * st + p0, nv, Xb1[s]);
    load_v<FULL, double, V>(a.Xb0 + s * st + p0, nv, Xb0in[s]);
    if (a.taubar) load_v<FULL, double, V>(a.taubar + s * st + p0, nv, tb[s]);
    else
#pragma unroll
      for (int v = 0; v < V; ++v) tb[s][v] = 0.0;
  }
  double kbar[D * D][V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
#pragma unroll
    for (int t = 0; t < D * D; ++t) kbar[t][v] = 0.0;
    if (!(FULL || v < nv)) continue;
    double k[D * D], S[C], x0[C], x1[C], x2[C], x1b[C], x2b[C], tv[C];
#pragma unroll
    for (int t = 0; t < D * D; ++t) k[t] = kt[t][v];
#pragma unroll
    for (int s = 0; s < C; ++s) {
      const int i = Sym<D>::i(s), j = Sym<D>::j(s);
      S[s] = k[i * D + j] + k[j * D + i];
      x0[s] = X0[s][v]; x1[s] = X1[s][v]; x2[s] = X2[s][v];
      tv[s] = tb[s][v];
      // tau^1 = gamma (theta X^(2) - hr X^(1));  X^1 = X^(2)
      x2b[s] = X2b[s][v] + Xb1[s][v] + a.s.gamma * a.s.theta * tv[s];
      x1b[s] = X1b[s][v] - a.s.gamma * a.s.hr * tv[s];
    }
    double scale_g = 0.0;
#pragma unroll
    for (int s = 0; s < C; ++s) scale_g += tv[s] * (a.s.theta * x2[s] - a.s.hr * x1[s]);
    sc[5] += scale_g;                               // gamma
    sc[6] += a.s.gamma * dot<C>(tv, x2);            // theta
    sc[7] += -a.s.gamma * dot<C>(tv, x1);           // hr
    double M[C][C], rb[C], Kx[C], kb_[D * D];
#pragma unroll
    for (int t = 0; t < D * D; ++t) kb_[t] = 0.0;
    const double idv = SP ? a.s.inv_De + rate[v] : a.s.inv_De;
    const double s1 = SP ? a.s.src1 * srcw[v] : a.s.src1;
    const double s2 = SP ? a.s.sigma2 * srcw[v] : a.s.sigma2;
    double didv = 0.0;                              // dL/d(1/De + rate) of this point
    const double diag1 = 1.0 + a.s.hgt * idv;
    // stage 2: M X^(2) = X^0 + sigma1 A(X^(1)) + sigma2 S
    build_M<D>(k, diag1, a.s.hgt, M);
#pragma unroll
    for (int s = 0; s < C; ++s) rb[s] = x2b[s];
    solve_transposed<C>(M, rb);
    apply_K<D>(k, x2, Kx);
    const double rx2 = dot<C>(rb, x2);
    sc[1] += -rx2 * idv + dot<C>(rb, Kx);          // hgt (matrix)
    sc[0] += -rx2 * a.s.hgt;                        // 1/De (matrix)
    didv += -rx2 * a.s.hgt;
    kgrad_VZ<D>(kb_, a.s.hgt, rb, x2);
    double AX[C];
    apply_K<D>(k, x1, AX);
#pragma unroll
    for (int s = 0; s < C; ++s) AX[s] -= idv * x1[s];
    sc[3] += dot<C>(rb, AX);                        // sigma1
    sc[4] += (SP ? srcw[v] : 1.0) * dot<C>(rb, S);  // sigma2
    kgrad_V<D>(kb_, s2, rb);
    double x0b[C];
#pragma unroll
    for (int s = 0; s < C; ++s) x0b[s] = X0b[s][v] + rb[s];
    // A(X^(1)) = K X^(1) - X^(1)/De with adjoint sigma1 Rbar2
    double axb[C], Km[C][C];
#pragma unroll
    for (int s = 0; s < C; ++s) axb[s] = a.s.sigma1 * rb[s];
    build_K<D>(k, Km);
#pragma unroll
    for (int t = 0; t < C; ++t) {
      double acc = 0.0;
#pragma unroll
      for (int s = 0; s < C; ++s) acc += Km[s][t] * axb[s];
      x1b[t] += acc - idv * axb[t];
    }
    sc[0] += -dot<C>(axb, x1);                      // 1/De
    didv += -dot<C>(axb, x1);
    kgrad_VZ<D>(kb_, 1.0, axb, x1);
    // stage 1: M X^(1) = X^0 + src1 S
    build_M<D>(k, diag1, a.s.hgt, M);
#pragma unroll
    for (int s = 0; s < C; ++s) rb[s] = x1b[s];
    solve_transposed<C>(M, rb);
    apply_K<D>(k, x1, Kx);
    const double rx1 = dot<C>(rb, x1);
    sc[1] += -rx1 * idv + dot<C>(rb, Kx);
    sc[0] += -rx1 * a.s.hgt;
    didv += -rx1 * a.s.hgt;
    if constexpr (SP) sc[8] += rate[v] * didv;     // rate through 1/De + rate
    kgrad_VZ<D>(kb_, a.s.hgt, rb, x1);
    sc[2] += (SP ? srcw[v] : 1.0) * dot<C>(rb, S);  // src1
    kgrad_V<D>(kb_, s1, rb);
#pragma unroll
    for (int s = 0; s < C; ++s) X0b[s][v] = Xb0in[s][v] + x0b[s] + rb[s];
#pragma unroll
    for (int t = 0; t < D * D; ++t) kbar[t][v] = kb_[t];
  }
#pragma unroll
  for (int s = 0; s < C; ++s) store_v<FULL, double, V>(a.Xb0 + s * st + p0, nv, X0b[s]);
  if (a.kba) {
#pragma unroll
    for (int t = 0; t < D * D; ++t) {
      double x[V];
      load_v<FULL, double, V>(a.kba + t * st + p0, nv, x);
#pragma unroll
      for (int v = 0; v < V; ++v) x[v] += kbar[t][v];
      store_v<FULL, double, V>(a.kba + t * st + p0, nv, x);
    }
  }
}

template <int D, typename MT, typename KT, int V, bool SP>
__global__ __launch_bounds__(kBlock) void start_adj_kernel(const StartAdjArgs<MT, KT> a) {
  extern __shared__ double smode[];
  for (int j = threadIdx.x; j < (kBlock / 64) * 3 * a.m; j += kBlock) smode[j] = 0.0;
  __syncthreads();
  double sc[kNumAdjScalars];
#pragma unroll
  for (int i = 0; i < kNumAdjScalars; ++i) sc[i] = 0.0;
  const int64_t ngroups = (a.npts + V - 1) / V;
  const int64_t gstride = (int64_t)gridDim.x * kBlock;
  for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x - (threadIdx.x % 64); g < ngroups; g += gstride) {
    const int64_t mine = g + (threadIdx.x % 64);
    const int64_t p0 = mine * V;
    int nv = (int)((a.npts - p0) < V ? (a.npts - p0) : V);
    if (mine >= ngroups) nv = 0;
    if (nv == V) start_adj_group<D, MT, KT, V, true, SP>(a, p0, nv, smode, sc);
    else start_adj_group<D, MT, KT, V, false, SP>(a, nv > 0 ? p0 : 0, nv, smode, sc);
  }
  __syncthreads();
  write_block_partial(a.part, a.m, smode, sc);
}

// One block per entry of the partial vector: sums the block partials in order and adds the
// result to pbar at that entry's position (dest[j] >= 0), or at zeta_dest (dest[j] == -2).
__global__ __launch_bounds__(kBlock) void adj_finish_kernel(const double* __restrict__ part, int nparts, int np,
                                                            const int* __restrict__ dest, int64_t zeta_dest,
                                                            double* __restrict__ pbar) {
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kBlock) s += part[(size_t)b * np + j];
  __shared__ double sh[kBlock / 64];
  s = wave_sum(s);
  if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
    if (dest[j] >= 0) pbar[dest[j]] += t;
    else if (dest[j] == -2) pbar[zeta_dest] += t;
  }
}

// ------------------------------------------------------------------ dispatch
int grid_adj(const tfs_plan_s* p, int64_t ngroups) {
  const int64_t cap = (int64_t)p->num_cus * p->grid_per_cu;
  int64_t g = (ngroups + kBlock - 1) / kBlock;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

size_t adj_shared_bytes(const tfs_plan_s* p, int V) {
  const int ns = p->d == 2 ? AdjSlots<2>::N : AdjSlots<3>::N;
  return sizeof(double) * ((size_t)(kBlock / 64) * 3 * p->m + (size_t)ns * V * kBlock);
}

// Whole waves of V-point groups with the V-wide kernel, the remaining points (fewer than
// 64 V) with the masked V = 1 kernel; one finisher folds the block partials of both.
template <int D, typename MT, typename KT, int V, bool SP, bool ZF>
hipError_t adj_go_(const tfs_plan_s* p, AdjArgs<MT, KT> a, int64_t zeta_dest, double* pbar) {
  const int64_t nwaves = p->npoints / (64 * V);
  const int64_t p_tail = nwaves * 64 * V, rest = p->npoints - p_tail;
  int nb = 0, nt = 0;
  if (nwaves > 0) {
    a.p_begin = 0;
    a.ngroups = nwaves * 64;
    a.part0 = 0;
    nb = grid_adj(p, a.ngroups);
    const size_t shm = adj_shared_bytes(p, V);
    if (shm > 65536) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&adj_kernel<D, MT, KT, V, true, SP, ZF>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((adj_kernel<D, MT, KT, V, true, SP, ZF>), dim3(nb), dim3(kBlock), shm, p->stream, a);
  }
  if (rest > 0) {
    a.p_begin = p_tail;
    a.ngroups = rest;
    a.part0 = nb;
    nt = grid_adj(p, rest);
    hipLaunchKernelGGL((adj_kernel<D, MT, KT, 1, false, SP, ZF>), dim3(nt), dim3(kBlock), adj_shared_bytes(p, 1),
                       p->stream, a);
  }
  const int np = 3 * p->m + kNumAdjScalars;
  hipLaunchKernelGGL(adj_finish_kernel, dim3(np), dim3(kBlock), 0, p->stream, a.part, nb + nt, np,
                     p->d_dest_bdf2, zeta_dest, pbar);
  return hipGetLastError();
}

// The spatial form reads FP64 velocity gradients only (an FP32-kappa plan refuses it).
template <int D, typename MT, typename KT, int V, bool ZF>
hipError_t adj_go_z(const tfs_plan_s* p, const AdjArgs<MT, KT>& a, int64_t zeta_dest, double* pbar) {
  if constexpr (sizeof(KT) == 8) {
    if (a.sp.rate || a.sp.src >= 0) return adj_go_<D, MT, KT, V, true, ZF>(p, a, zeta_dest, pbar);
  }
  return adj_go_<D, MT, KT, V, false, ZF>(p, a, zeta_dest, pbar);
}

template <int D, typename MT, typename KT, int V>
hipError_t adj_go(const tfs_plan_s* p, const AdjArgs<MT, KT>& a, int64_t zeta_dest, double* pbar) {
  return p->zform ? adj_go_z<D, MT, KT, V, true>(p, a, zeta_dest, pbar)
                  : adj_go_z<D, MT, KT, V, false>(p, a, zeta_dest, pbar);
}

template <int D, typename MT, typename KT, int V>
hipError_t start_adj_go(const tfs_plan_s* p, const StartAdjArgs<MT, KT>& a, double* pbar) {
  const int64_t ngroups = (a.npts + V - 1) / V;
  const int grid = grid_adj(p, ngroups);
  const size_t shm = sizeof(double) * (kBlock / 64) * 3 * p->m;
  bool sp = false;
  if constexpr (sizeof(KT) == 8) sp = a.sp.rate || a.sp.src >= 0;
  if (sp) {
    if constexpr (sizeof(KT) == 8)
      hipLaunchKernelGGL((start_adj_kernel<D, MT, KT, V, true>), dim3(grid), dim3(kBlock), shm, p->stream, a);
  } else {
    hipLaunchKernelGGL((start_adj_kernel<D, MT, KT, V, false>), dim3(grid), dim3(kBlock), shm, p->stream, a);
  }
  const int np = 3 * p->m + kNumAdjScalars;
  hipLaunchKernelGGL(adj_finish_kernel, dim3(np), dim3(kBlock), 0, p->stream, a.part, grid, np,
                     p->d_dest_start, (int64_t)-1, pbar);
  return hipGetLastError();
}

bool al(const void* ptr, size_t b) { return ptr == nullptr || ((uintptr_t)ptr % b) == 0; }

// Points per lane of the BDF2 adjoint: the "adj_vec" tuning (0 = default 1), if every field
// is aligned for it and its LDS slots fit in 64 KB per block.
template <typename MT, typename KT>
int adj_vec(const tfs_plan_s* p, const AdjLevels& L) {
  const int want = p->adj_vec_override ? p->adj_vec_override : (sizeof(MT) == 4 ? 2 : 1);
  const int V = want == 2 ? 2 : 1;
  if (V == 1) return 1;
  if (p->stride % V || p->tile % V || adj_shared_bytes(p, V) > (size_t)p->lds_max) return 1;
  const size_t bm = (size_t)V * sizeof(MT), bd = (size_t)V * 8, bk = (size_t)V * sizeof(KT);
  if (al(L.ka, bk) && al(L.kb, bk) && al(L.Xn, bd) && al(L.Xm, bd) && al(L.Xmm, bd) && al(L.Xp, bd) && al(L.Xbar, bd) &&
      al(L.taubar, bd) && al(L.kba, bd) && al(L.kbb, bd) && al(L.Yn, bm) && al(L.Ym, bm) && al(L.Hbar, bm))
    return V;
  return 1;
}

size_t exp_adj_shared_bytes(const tfs_plan_s* p, int V) {
  return sizeof(double) * ((size_t)(kBlock / 64) * 3 * p->m + (size_t)p->c * V * kBlock);
}

template <int D, typename MT, typename KT, int V, bool TAU, bool SP>
hipError_t exp_adj_go_(const tfs_plan_s* p, ExpAdjArgs<MT, KT> a, int64_t zeta_dest, double* pbar) {
  const int64_t nwaves = p->npoints / (64 * V);
  const int64_t p_tail = nwaves * 64 * V, rest = p->npoints - p_tail;
  int nb = 0, nt = 0;
  if (nwaves > 0) {
    a.p_begin = 0;
    a.ngroups = nwaves * 64;
    a.part0 = 0;
    nb = grid_adj(p, a.ngroups);
    const size_t shm = exp_adj_shared_bytes(p, V);
    if (shm > 65536) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&exp_adj_kernel<D, MT, KT, V, true, TAU, SP>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((exp_adj_kernel<D, MT, KT, V, true, TAU, SP>), dim3(nb), dim3(kBlock), shm, p->stream, a);
  }
  if (rest > 0) {
    a.p_begin = p_tail;
    a.ngroups = rest;
    a.part0 = nb;
    nt = grid_adj(p, rest);
    hipLaunchKernelGGL((exp_adj_kernel<D, MT, KT, 1, false, TAU, SP>), dim3(nt), dim3(kBlock), exp_adj_shared_bytes(p, 1),
                       p->stream, a);
  }
  const int np = 3 * p->m + kNumAdjScalars;
  hipLaunchKernelGGL(adj_finish_kernel, dim3(np), dim3(kBlock), 0, p->stream, a.part, nb + nt, np,
                     p->d_dest_exp, zeta_dest, pbar);
  return hipGetLastError();
}

template <int D, typename MT, typename KT, int V>
hipError_t exp_adj_go(const tfs_plan_s* p, const ExpAdjArgs<MT, KT>& a, int64_t zeta_dest, double* pbar) {
  if constexpr (sizeof(KT) == 8) {
    if (a.sp.rate || a.sp.src >= 0)
      return a.taubar ? exp_adj_go_<D, MT, KT, V, true, true>(p, a, zeta_dest, pbar)
                      : exp_adj_go_<D, MT, KT, V, false, true>(p, a, zeta_dest, pbar);
  }
  return a.taubar ? exp_adj_go_<D, MT, KT, V, true, false>(p, a, zeta_dest, pbar)
                  : exp_adj_go_<D, MT, KT, V, false, false>(p, a, zeta_dest, pbar);
}

template <int D, typename MT, typename KT>
hipError_t exp_adj_dispatch(const tfs_plan_s* p, int64_t n, const AdjLevels& L, double* pbar) {
  const int64_t st = p->stride;
  const int64_t xs = (int64_t)Sym<D>::C * st;
  const int sn = (int)(n % 2), sp = 1 - sn;
  ExpAdjArgs<MT, KT> a;
  a.ka = static_cast<const KT*>(L.ka);
  a.kb = n >= 1 ? static_cast<const KT*>(L.kb) : nullptr;
  a.Xn = L.Xn;
  a.Xp = L.Xp;
  a.Yn = static_cast<const MT*>(L.Yn);
  a.Xb_in = L.Xbar + sp * xs;
  a.Xb_out = L.Xbar + sn * xs;
  a.H = static_cast<MT*>(L.Hbar);
  a.taubar = L.taubar;
  a.kba = L.kba;
  a.kbb = L.kbb;
  a.kb_same = (L.kba != nullptr && L.kba == L.kbb) ? 1 : 0;
  a.coef = p->d_coef;
  a.part = p->d_adj_part;
  a.stride = st;
  a.tile = p->tile;
  a.m = p->m;
  a.s.a_diag = 1.0 + p->q_e / p->De;
  a.s.q = p->q_e;
  a.s.s_h = p->s_h;
  a.s.inv_De = 1.0 / p->De;
  a.s.zeta = p->zeta[n + 1];
  a.s.tau_scale = p->tau_scale;
  a.s.eta_e = p->eta_e;
  a.s.fa = 1.5;
  a.s.fb = -0.5;
  a.s.first = n == 0 ? 1 : 0;
  a.dt = p->dt;
  a.sp.rate = p->sp_rate;
  a.sp.src = p->sp_source;
  const int64_t zd = (int64_t)kPbarScalars + 6 * p->m + n + 1;
  // one point per lane unless tuned: measured faster than two for this kernel
  const int want = p->adj_vec_override ? p->adj_vec_override : 1;
  bool two = want == 2 && p->stride % 2 == 0 && p->tile % 2 == 0 && exp_adj_shared_bytes(p, 2) <= (size_t)p->lds_max;
  const size_t bm = 2 * sizeof(MT), bd = 16, bk = 2 * sizeof(KT);
  two = two && al(L.ka, bk) && al(L.kb, bk) && al(L.Xn, bd) && al(L.Xp, bd) && al(L.Xbar, bd) &&
        al(L.taubar, bd) && al(L.kba, bd) && al(L.kbb, bd) && al(L.Yn, bm) && al(L.Hbar, bm);
  if (two) return exp_adj_go<D, MT, KT, 2>(p, a, zd, pbar);
  return exp_adj_go<D, MT, KT, 1>(p, a, zd, pbar);
}

template <int D, typename MT, typename KT>
hipError_t adj_dispatch(const tfs_plan_s* p, int64_t n, const AdjLevels& L, double* pbar) {
  const int64_t st = p->stride;
  const int64_t ys = (int64_t)p->m * Sym<D>::C * st;
  const int64_t xs = (int64_t)Sym<D>::C * st;
  const int sn = (int)(n % 2), sp = 1 - sn;
  MT* Hb = static_cast<MT*>(L.Hbar);
  if (n == 0) {
    StartAdjArgs<MT, KT> a;
    a.ka = static_cast<const KT*>(L.ka);
    a.X0 = L.Xn;
    a.Xb0 = L.Xbar;
    a.Xb1 = L.Xbar + xs;
    a.H1 = Hb + ys;
    a.H2 = Hb;
    a.taubar = L.taubar;
    a.kba = L.kba;
    a.coef = p->d_coef;
    a.part = p->d_adj_part;
    a.npts = p->npoints;
    a.stride = st;
    a.tile = p->tile;
    a.m = p->m;
    a.zform = p->zform ? 1 : 0;
    a.s.hgt = p->hg * p->theta;
    a.s.inv_De = 1.0 / p->De;
    a.s.src1 = p->hg * p->theta;
    a.s.sigma1 = p->sigma1;
    a.s.sigma2 = p->sigma2;
    a.s.gamma = p->gamma;
    a.s.theta = p->theta;
    a.s.hr = p->hr;
    a.sp.rate = p->sp_rate;
    a.sp.src = p->sp_source;
    return start_adj_go<D, MT, KT, 1>(p, a, pbar);
  }
  AdjArgs<MT, KT> a;
  a.ka = static_cast<const KT*>(L.ka);
  a.kb = static_cast<const KT*>(L.kb);
  a.Xn = L.Xn;
  a.Xm = L.Xm;
  a.Xmm = p->zform ? L.Xmm : nullptr;
  a.Xp = L.Xp;
  a.Yn = static_cast<const MT*>(L.Yn);
  a.Ym = static_cast<const MT*>(L.Ym);
  if (p->zform) {
    a.Xb_new = L.Xbar + ((n + 1) % 3) * xs;
    a.Xb_cur = L.Xbar + (n % 3) * xs;
    a.Xb_old = L.Xbar + ((n - 1) % 3) * xs;
  } else {
    a.Xb_new = L.Xbar + sp * xs;
    a.Xb_cur = L.Xbar + sn * xs;
    a.Xb_old = nullptr;
  }
  a.H1 = Hb + sp * ys;
  a.H2 = Hb + sn * ys;
  a.taubar = L.taubar;
  a.kba = L.kba;
  a.kbb = L.kbb;
  a.kb_same = (L.kba != nullptr && L.kba == L.kbb) ? 1 : 0;
  a.coef = p->d_coef;
  a.part = p->d_adj_part;
  a.stride = st;
  a.tile = p->tile;
  a.m = p->m;
  a.s.a_diag = p->a_diag;
  a.s.eta = p->eta;
  a.s.s_ec = p->s_ec;
  a.s.inv_De = 1.0 / p->De;
  a.s.zeta = p->zeta[n + 1];
  a.s.tau_scale = p->tau_scale;
  a.sp.rate = p->sp_rate;
  a.sp.src = p->sp_source;
  // the zeta gradient of this step goes to pbar[zeta offset + n + 1]
  const int64_t zd = (int64_t)kPbarScalars + 6 * p->m + n + 1;
  if (adj_vec<MT, KT>(p, L) == 2) return adj_go<D, MT, KT, 2>(p, a, zd, pbar);
  return adj_go<D, MT, KT, 1>(p, a, zd, pbar);
}

}  // namespace

// The plan's (dim, mode precision, kappa precision) instance of a dispatcher; FP32 velocity
// gradients exist only with FP32 modes.
#define TFS_ADJ_DISPATCH(fn)                                                                        \
  (p->precision == TFS_FP64                                                                         \
       ? (p->d == 2 ? fn<2, double, double>(p, n, L, pbar) : fn<3, double, double>(p, n, L, pbar)) \
       : p->kappa_f32                                                                               \
             ? (p->d == 2 ? fn<2, float, float>(p, n, L, pbar) : fn<3, float, float>(p, n, L, pbar))  \
             : (p->d == 2 ? fn<2, float, double>(p, n, L, pbar) : fn<3, float, double>(p, n, L, pbar)))

hipError_t launch_adjoint(const tfs_plan_s* p, int64_t n, const AdjLevels& L, double* pbar) {
  if (p->npoints == 0) return hipSuccess;
  if (p->scheme == TFS_SCHEME_EXP) return TFS_ADJ_DISPATCH(exp_adj_dispatch);
  return TFS_ADJ_DISPATCH(adj_dispatch);
}

}  // namespace tfs

// Host side of the C ABI: plan validation, FP64 coefficient tables, the mass-mode
// memory table, the sum-of-exponentials fit, and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "tfs_internal.h"

namespace {

thread_local std::string g_last_error;

tfs_status fail(tfs_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

tfs_status hip_fail(hipError_t e, const char* what) {
  return fail(TFS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool finite_nonneg(double x) { return std::isfinite(x) && x >= 0.0; }

// Neumaier-compensated accumulator.
struct CompSum {
  double s = 0.0, c = 0.0;
  void add(double x) {
    double t = s + x;
    if (std::fabs(s) >= std::fabs(x)) c += (s - t) + x; else c += (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

// Legendre P_n(z) and P_{n-1}(z) by the three-term recurrence.
void legendre_pair(int n, double z, double* pn, double* pnm1) {
  double a = 1.0, b = z;  // P_0, P_1
  if (n == 0) { *pn = 1.0; *pnm1 = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    const double c = ((2.0 * k - 1.0) * z * b - (k - 1.0) * a) / k;
    a = b;
    b = c;
  }
  *pn = b;
  *pnm1 = a;
}

// Gauss-Legendre nodes (ascending) and weights on [-1, 1]: Newton iteration on P_n from
// the asymptotic node guesses; P_n'(z) = n (P_{n-1}(z) - z P_n(z)) / (1 - z^2),
// weight 2 / ((1 - z^2) P_n'(z)^2).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& wq) {
  x.assign(n, 0.0);
  wq.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double pn, pnm1, dp;
    for (int it = 0; it < 100; ++it) {
      legendre_pair(n, z, &pn, &pnm1);
      dp = n * (pnm1 - z * pn) / (1.0 - z * z);
      const double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) <= 1e-16 * std::max(1.0, std::fabs(z))) break;
    }
    legendre_pair(n, z, &pn, &pnm1);
    dp = n * (pnm1 - z * pn) / (1.0 - z * z);
    x[n - 1 - i] = z;
    wq[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

void soe_rule(double alpha, int m, double ylo, double yhi, double* w, double* lam, double* dw,
              double* dlam) {
  for (int k = 0; k < m; ++k) {
    w[k] = 0.0; lam[k] = 0.0;
    if (dw) dw[k] = 0.0;
    if (dlam) dlam[k] = 0.0;
  }
  if (alpha == 1.0) {
    w[0] = 1.0;
    return;
  }
  const double s = std::sin(M_PI * alpha) / M_PI;
  const double cot = M_PI * std::cos(M_PI * alpha) / std::sin(M_PI * alpha);
  w[0] = s * std::exp((1.0 - alpha) * ylo) / (1.0 - alpha);
  if (dw) dw[0] = w[0] * (cot - ylo + 1.0 / (1.0 - alpha));
  if (m >= 2) {
    const int j = m - 1;
    lam[j] = std::exp(yhi) * (1.0 + alpha) / alpha;
    w[j] = s * std::exp((1.0 - alpha) * yhi) * (1.0 + alpha) / (alpha * alpha);
    if (dlam) dlam[j] = -std::exp(yhi) / (alpha * alpha);
    if (dw) dw[j] = w[j] * (cot - yhi + 1.0 / (1.0 + alpha) - 2.0 / alpha);
  }
  if (m >= 3) {
    std::vector<double> x, gw;
    gauss_legendre(m - 2, x, gw);
    const double half = 0.5 * (yhi - ylo), mid = 0.5 * (yhi + ylo);
    for (int i = 0; i < m - 2; ++i) {
      const double y = mid + half * x[i];
      w[1 + i] = s * half * gw[i] * std::exp((1.0 - alpha) * y);
      lam[1 + i] = std::exp(y);
      if (dw) dw[1 + i] = w[1 + i] * (cot - y);
    }
  }
}

// Exact one-step weights of a mode for X linear on the step (TFS_SCHEME_EXP), z = lambda dt:
// e = exp(-z), om = 1 - e, a0 = (om - z e)/z^2, a1 = (z - om)/z^2.  Below z = 0.1 the
// quotients lose digits, so a0 and a1 come from their Taylor series there,
// a0 = sum_j (-z)^j (j+1)/(j+2)!, a1 = sum_j (-z)^j/(j+2)!, summed from the small end.
void exp_mode_weights(double z, double* e, double* om, double* a0, double* a1, double* b2 = nullptr) {
  *e = std::exp(-z);
  *om = -std::expm1(-z);
  if (z < 0.1) {
    double fac[26];
    fac[0] = 1.0;
    for (int j = 1; j < 26; ++j) fac[j] = fac[j - 1] * j;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int j = 21; j >= 0; --j) {
      const double zj = std::pow(-z, j);
      s0 += zj * (j + 1) / fac[j + 2];
      s1 += zj / fac[j + 2];
      s2 += zj * (j + 1) * (j + 2) / fac[j + 3];
    }
    *a0 = s0;
    *a1 = s1;
    if (b2) *b2 = s2;
  } else {
    *a0 = (*om - z * *e) / (z * z);
    *a1 = (z - *om) / (z * z);
    // b2 = int_0^1 v^2 e^{-zv} dv = (2 om - 2 z e - z^2 e) / z^3  (= -d a0 / dz)
    if (b2) *b2 = (2.0 * *om - z * *e * (2.0 + z)) / (z * z * z);
  }
}

double symbol_relerr(double alpha, int m, const double* w, const double* lam, double dt, double T, int ns) {
  const double lo = std::log(0.1 / T), hi = std::log(10.0 / dt);
  double worst = 0.0;
  for (int i = 0; i < ns; ++i) {
    const double s = std::exp(lo + (hi - lo) * i / (ns - 1));
    double K = 0.0;
    for (int k = 0; k < m; ++k) K += w[k] / (s + lam[k]);
    worst = std::max(worst, std::fabs(K * std::pow(s, alpha) - 1.0));
  }
  return worst;
}

double kernel_relerr(double alpha, int m, const double* w, const double* lam, double dt, double T, int ns) {
  const double lo = std::log(dt), hi = std::log(T);
  const double g = std::tgamma(alpha);
  double worst = 0.0;
  for (int i = 0; i < ns; ++i) {
    const double t = std::exp(lo + (hi - lo) * i / (ns - 1));
    double K = 0.0;
    for (int k = 0; k < m; ++k) K += w[k] * std::exp(-lam[k] * t);
    const double ex = std::pow(t, alpha - 1.0) / g;
    worst = std::max(worst, std::fabs(K - ex) / ex);
  }
  return worst;
}

// The plan runs the spatial form (tfs_plan_set_spatial).
bool spatial(const tfs_plan_s* p) { return p->sp_rate != nullptr || p->sp_source >= 0; }

}  // namespace

namespace tfs {
// Error reporting for the other translation units of the library (the coupled step).
tfs_status set_error(tfs_status s, const char* msg) { return fail(s, "%s", msg); }
}  // namespace tfs

extern "C" {

const char* tfs_last_error(void) { return g_last_error.c_str(); }

const char* tfs_status_string(tfs_status s) {
  switch (s) {
    case TFS_OK: return "ok";
    case TFS_EINVAL: return "invalid argument";
    case TFS_ENOMEM: return "out of memory";
    case TFS_EHIP: return "HIP runtime error";
    case TFS_ENUMERIC: return "non-finite or non-positive-definite state";
    case TFS_EUNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

tfs_status tfs_soe_gl_log(double alpha, int32_t m, double y_lo, double y_hi, double* w, double* lambda,
                          double* dw_dalpha, double* dlambda_dalpha) {
  if (!(alpha > 0.0 && alpha <= 1.0)) return fail(TFS_EINVAL, "alpha must be in (0, 1]");
  if (m < 1) return fail(TFS_EINVAL, "m must be >= 1");
  if (!w || !lambda) return fail(TFS_EINVAL, "null output");
  if (!(y_lo < y_hi) || !std::isfinite(y_lo) || !std::isfinite(y_hi))
    return fail(TFS_EINVAL, "need finite y_lo < y_hi");
  soe_rule(alpha, m, y_lo, y_hi, w, lambda, dw_dalpha, dlambda_dalpha);
  return TFS_OK;
}

tfs_status tfs_soe_fit(double alpha, int32_t m, double dt, double T, double* w, double* lambda,
                       double* dw_dalpha, double* dlambda_dalpha, double* info) {
  if (!(alpha > 0.0 && alpha <= 1.0)) return fail(TFS_EINVAL, "alpha must be in (0, 1]");
  if (m < 1) return fail(TFS_EINVAL, "m must be >= 1");
  if (!(dt > 0.0) || !(T > dt)) return fail(TFS_EINVAL, "need 0 < dt < T");
  if (!w || !lambda) return fail(TFS_EINVAL, "null output");
  if (alpha == 1.0) {
    soe_rule(alpha, m, 0.0, 1.0, w, lambda, dw_dalpha, dlambda_dalpha);
    if (info) { info[0] = 0.0; info[1] = 1.0; info[2] = 0.0; info[3] = 0.0; }
    return TFS_OK;
  }
  std::vector<double> ww(m), ll(m);
  const double lo0 = std::log(0.1 / T), hi0 = std::log(10.0 / dt);
  double best = std::numeric_limits<double>::infinity(), blo = lo0, bhi = hi0;
  // coarse search over the window, then a fine search around the best cell
  for (int i = 0; i <= 34; ++i) {
    for (int j = 0; j <= 42; ++j) {
      const double ylo = lo0 - 16.0 + 0.5 * i, yhi = hi0 - 2.0 + 1.0 * j;
      soe_rule(alpha, m, ylo, yhi, ww.data(), ll.data(), nullptr, nullptr);
      const double e = symbol_relerr(alpha, m, ww.data(), ll.data(), dt, T, 120);
      if (e < best) { best = e; blo = ylo; bhi = yhi; }
    }
  }
  const double clo = blo, chi = bhi;
  for (int i = 0; i <= 10; ++i) {
    for (int j = 0; j <= 20; ++j) {
      const double ylo = clo - 0.5 + 0.1 * i, yhi = chi - 1.0 + 0.1 * j;
      soe_rule(alpha, m, ylo, yhi, ww.data(), ll.data(), nullptr, nullptr);
      const double e = symbol_relerr(alpha, m, ww.data(), ll.data(), dt, T, 120);
      if (e < best) { best = e; blo = ylo; bhi = yhi; }
    }
  }
  soe_rule(alpha, m, blo, bhi, w, lambda, dw_dalpha, dlambda_dalpha);
  if (info) {
    info[0] = blo;
    info[1] = bhi;
    info[2] = symbol_relerr(alpha, m, w, lambda, dt, T, 300);
    info[3] = kernel_relerr(alpha, m, w, lambda, dt, T, 400);
  }
  return TFS_OK;
}

tfs_status tfs_plan_create(const tfs_plan_desc* desc, tfs_plan* out) {
  if (!out) return fail(TFS_EINVAL, "null output plan pointer");
  *out = nullptr;
  if (!desc) return fail(TFS_EINVAL, "null descriptor");
  const tfs_plan_desc& D = *desc;
  if (D.dim != 2 && D.dim != 3) return fail(TFS_EINVAL, "dim must be 2 or 3 (got %d)", D.dim);
  if (D.nmodes < 1 || D.nmodes > tfs::kMaxModes)
    return fail(TFS_EINVAL, "nmodes must be in [1, %d]", tfs::kMaxModes);
  if (D.npoints < 0) return fail(TFS_EINVAL, "npoints must be >= 0");
  if (D.tile < 0 || D.tile % 4 != 0) return fail(TFS_EINVAL, "tile must be 0 or a positive multiple of 4");
  int64_t stride = D.stride;
  if (stride == 0) stride = D.tile > 0 ? (D.npoints + D.tile - 1) / D.tile * D.tile : D.npoints;
  if (stride < D.npoints) return fail(TFS_EINVAL, "stride must be >= npoints");
  if (D.tile > 0 && stride % D.tile != 0) return fail(TFS_EINVAL, "stride must be a multiple of tile");
  if (D.tile > 0 && D.tile < stride) {
    // lanes address the mode layout by 32-bit byte offsets from their wave's first point,
    // which may lie one tile earlier
    const double span = ((double)D.nmodes * (D.dim * (D.dim + 1) / 2) * (double)(D.tile + 256) + 256.0) * 8.0;
    if (span >= 2147483648.0) return fail(TFS_EINVAL, "tile too large for nmodes (tile * nmodes * c * 8 >= 2^31)");
  }
  if (!(D.alpha > 0.0 && D.alpha <= 1.0)) return fail(TFS_EINVAL, "alpha must be in (0, 1]");
  if (!(D.De > 0.0) || !std::isfinite(D.De)) return fail(TFS_EINVAL, "De must be > 0");
  if (!(D.eta_p >= 0.0) || !std::isfinite(D.eta_p)) return fail(TFS_EINVAL, "eta_p must be >= 0");
  if (!(D.dt > 0.0) || !std::isfinite(D.dt)) return fail(TFS_EINVAL, "dt must be > 0");
  if (D.max_steps < 1) return fail(TFS_EINVAL, "max_steps must be >= 1");
  if (!D.w || !D.lambda) return fail(TFS_EINVAL, "null w or lambda");
  if (D.precision != TFS_FP64 && D.precision != TFS_FP32_MODES) return fail(TFS_EINVAL, "unknown precision");
  if (D.scheme != TFS_SCHEME_BDF2 && D.scheme != TFS_SCHEME_EXP) return fail(TFS_EINVAL, "unknown scheme");
  if (D.kappa_precision != TFS_KAPPA_FP64 && D.kappa_precision != TFS_KAPPA_FP32)
    return fail(TFS_EINVAL, "unknown kappa precision");
  if (D.kappa_precision == TFS_KAPPA_FP32 && D.precision != TFS_FP32_MODES)
    return fail(TFS_EINVAL, "FP32 velocity gradients need an FP32-mode plan");
  if (D.mode_form != TFS_MODE_FORM_AUTO && D.mode_form != TFS_MODE_FORM_Y && D.mode_form != TFS_MODE_FORM_Z)
    return fail(TFS_EINVAL, "unknown mode form");
  if (D.mode_form == TFS_MODE_FORM_Z && D.scheme != TFS_SCHEME_BDF2)
    return fail(TFS_EINVAL, "the shifted mode form is a form of the BDF2 scheme");
  for (int k = 0; k < D.nmodes; ++k)
    if (!finite_nonneg(D.w[k]) || !finite_nonneg(D.lambda[k]))
      return fail(TFS_EINVAL, "w and lambda must be finite and >= 0 (mode %d)", k);

  tfs_plan_s* p = new (std::nothrow) tfs_plan_s();
  if (!p) return fail(TFS_ENOMEM, "plan allocation");
  p->d = D.dim;
  p->c = D.dim * (D.dim + 1) / 2;
  p->m = D.nmodes;
  p->npoints = D.npoints;
  p->stride = stride;
  p->tile = D.tile > 0 ? D.tile : stride;
  p->max_steps = D.max_steps;
  p->alpha = D.alpha;
  p->De = D.De;
  p->eta_p = D.eta_p;
  p->dt = D.dt;
  p->gamma = D.eta_p / D.De;
  p->precision = D.precision;
  p->kappa_f32 = D.kappa_precision == TFS_KAPPA_FP32;
  p->scheme = D.scheme;
  p->zform = D.scheme == TFS_SCHEME_BDF2 &&
             (D.mode_form == TFS_MODE_FORM_Z || (D.mode_form == TFS_MODE_FORM_AUTO && D.precision == TFS_FP32_MODES));
  p->xlev = p->zform ? 3 : 2;
  p->flags = D.flags;
  p->stream = static_cast<hipStream_t>(D.stream);
  p->w.assign(D.w, D.w + D.nmodes);
  p->lam.assign(D.lambda, D.lambda + D.nmodes);

  const int m = p->m;
  const double dt = p->dt, b0 = tfs::kB0;
  const double gs = 1.0 - 1.0 / std::sqrt(2.0);
  const double hg = dt * gs;
  p->hg = hg;
  p->coef.assign((size_t)tfs::kNumCoefAll * m, 0.0);
  CompSum eta, s_ec, theta, rho;
  for (int k = 0; k < m; ++k) {
    const double wk = p->w[k], lk = p->lam[k];
    const double dk = 1.0 / (b0 + lk * dt);
    const double ck = wk * dt * dk;
    const double ek = lk * dt * dk;
    const double r = 1.0 / (1.0 + hg * lk);
    p->coef[tfs::kRowD * m + k] = dk;
    p->coef[tfs::kRowDC * m + k] = dk * ck;
    p->coef[tfs::kRowEta * m + k] = ek;
    p->coef[tfs::kRowC * m + k] = ck;
    // start-up modes: X_k^1 = [h(1-gs) w_k r X^(1) + h gs w_k X^(2)] r;  Y_k^1 = X_k^1 - c_k X^1
    p->coef[tfs::kRowU * m + k] = dt * (1.0 - gs) * wk * r * r;
    p->coef[tfs::kRowV * m + k] = hg * wk * r - ck;
    // shifted form: the quasi-static value of a mode that follows X is (w_k/lambda_k) X, of
    // which Y_k keeps (w_k/lambda_k - c_k) X.  Only modes that relax within the plan's
    // horizon (lambda_k max_steps dt >= 1) come near it; a slower mode stays far below it,
    // and shifting it would store a value (w_k/lambda_k) |X| much larger than the mode.
    if (p->zform && lk > 0.0 && lk * dt * (double)p->max_steps >= 1.0)
      p->coef[tfs::kRowBeta * m + k] = wk / lk - ck;
    eta.add(b0 * ck);
    s_ec.add(ek * ck);
    theta.add(wk * r);
    rho.add(lk * wk * r * r);
  }
  p->eta = eta.value();
  p->s_ec = s_ec.value();
  p->a_diag = b0 + p->eta / p->De;
  p->tau_scale = p->gamma / dt;
  p->theta = theta.value();
  p->rho = rho.value();
  p->sigma1 = dt * (1.0 - gs) * (p->theta - hg * p->rho);
  p->sigma2 = dt * p->theta - hg * dt * (1.0 - gs) * p->rho;
  p->hr = dt * (1.0 - gs) * p->rho;

  // Mass-mode memory: mu_k^0 = 0, mu_k^1 from the SDIRK2 stages with mass 1, then the
  // BDF2 push-forward mu_k^{n+1} = d_k (2 mu_k^n - mu_k^{n-1}/2) + c_k; the step n -> n+1
  // uses zeta^{n+1} = eta - sum_k eta_k (2 mu_k^n - mu_k^{n-1}/2).
  p->zeta.assign((size_t)p->max_steps + 1, 0.0);
  {
    std::vector<double> mu_m(m, 0.0), mu_n(m);
    for (int k = 0; k < m; ++k) {
      const double r = 1.0 / (1.0 + hg * p->lam[k]);
      mu_n[k] = (dt * (1.0 - gs) * p->w[k] * r + hg * p->w[k]) * r;
    }
    for (int64_t n = 1; n < p->max_steps; ++n) {
      CompSum acc;
      for (int k = 0; k < m; ++k) {
        const double h = 2.0 * mu_n[k] - 0.5 * mu_m[k];
        acc.add(p->coef[tfs::kRowEta * m + k] * h);
        mu_m[k] = mu_n[k];
        mu_n[k] = p->coef[tfs::kRowD * m + k] * h + p->coef[tfs::kRowC * m + k];
      }
      p->zeta[n + 1] = p->eta - acc.value();
    }
  }

  if (p->scheme == TFS_SCHEME_EXP) {
    // Exponential mode update: Y_k^{n+1} = e_k Y_k^n + f_k X^n with Y_k = X_k - q_k X;
    // the mass modes mu_k (of the constant 1) give zeta^{n+1} = sum_k (mu_k^{n+1} - mu_k^n).
    CompSum q, sh, ee;
    std::vector<double> e(m), om(m), a0(m), a1(m), b2(m);
    for (int k = 0; k < m; ++k) {
      const double wk = p->w[k], lk = p->lam[k];
      exp_mode_weights(lk * dt, &e[k], &om[k], &a0[k], &a1[k], &b2[k]);
      const double qk = wk * dt * a1[k], rk = wk * dt * a0[k];
      p->coef[tfs::kRowE * m + k] = e[k];
      p->coef[tfs::kRowF * m + k] = e[k] * qk + rk;
      p->coef[tfs::kRowLdt * m + k] = lk * dt;
      p->coef[tfs::kRowQ * m + k] = qk;
      p->coef[tfs::kRowOneME * m + k] = om[k];
      p->coef[tfs::kRowR * m + k] = rk;
      // d a0/dz = -b2, d a1/dz = -(a0 - b2); q = w dt a1, r = w dt a0, f = e q + r
      const double dq_dl = -wk * dt * dt * (a0[k] - b2[k]);
      const double dr_dl = -wk * dt * dt * b2[k];
      p->coef[tfs::kRowFW * m + k] = dt * (e[k] * a1[k] + a0[k]);
      p->coef[tfs::kRowFL * m + k] = -dt * e[k] * qk + e[k] * dq_dl + dr_dl;
      p->coef[tfs::kRowQW * m + k] = -dt * a1[k];
      p->coef[tfs::kRowQL * m + k] = -dq_dl;
      q.add(qk);
      sh.add(om[k] * qk - rk);
      ee.add(dt * (wk - lk * qk));
    }
    p->q_e = q.value();
    p->s_h = sh.value();
    p->eta_e = ee.value();
    p->eta = p->q_e;
    p->s_ec = p->s_h;
    p->a_diag = 1.0 + p->q_e / p->De;
    p->theta = p->rho = p->sigma1 = p->sigma2 = p->hr = 0.0;
    std::fill(p->zeta.begin(), p->zeta.end(), 0.0);
    std::vector<double> mu(m, 0.0);
    for (int64_t n = 0; n < p->max_steps; ++n) {
      CompSum inc;
      for (int k = 0; k < m; ++k) {
        const double next = e[k] * mu[k] + p->w[k] * dt * (a0[k] + a1[k]);
        inc.add(next - mu[k]);
        mu[k] = next;
      }
      p->zeta[n + 1] = inc.value();
    }
  }

  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { delete p; return hip_fail(e, "hipGetDevice"); }
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus > 0)
    p->num_cus = cus;
  // Blocks per CU of the grid-stride launches.  FP64 modes: one persistent block per CU (four
  // waves of 16-byte mode accesses per CU keep enough bytes in flight; more waves only add
  // streams: 1024^2, m = 32 at 0.75 -> 0.80 of 8 TB/s and 256^3, m = 40 at 0.75 -> 0.78 on
  // MI355X).  FP32 modes, whose lanes move half the bytes per access: 16, several resident
  // blocks per CU.
  p->grid_per_cu = p->precision == TFS_FP64 ? 1 : 16;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device) == hipSuccess && lds > 0)
    p->lds_max = lds;
  // the static scratch of tfs_step_noalloc on this device; a failed lookup only disables that
  // entry point
  p->scratch_err = (int)tfs::scratch_address(p->device, &p->d_scratch);
  if (p->scratch_err != (int)hipSuccess) p->d_scratch = nullptr;
  e = hipMalloc(&p->d_coef, sizeof(double) * p->coef.size());
  if (e != hipSuccess) { delete p; return fail(TFS_ENOMEM, "coefficient table: %s", hipGetErrorString(e)); }
  e = hipMemcpy(p->d_coef, p->coef.data(), sizeof(double) * p->coef.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) { (void)hipFree(p->d_coef); delete p; return hip_fail(e, "upload coefficients"); }
  p->part_cap = tfs::max_blocks(p);
  e = hipMalloc(&p->d_part, sizeof(double) * tfs::kNumDiag * (size_t)std::max(1, p->part_cap));
  if (e != hipSuccess) { (void)hipFree(p->d_coef); delete p; return fail(TFS_ENOMEM, "diagnostic scratch"); }
  // adjoint: block partials and the pbar position of every partial entry
  const int np = 3 * m + tfs::kNumAdjScalars;
  std::vector<int> dest_b(np, -1), dest_s(np, -1);
  for (int j = 0; j < 3 * m; ++j) { dest_b[j] = j; dest_s[j] = 3 * m + j; }
  const int sb = 6 * m;
  dest_b[3 * m + 0] = sb + tfs::kPbA;
  dest_b[3 * m + 1] = sb + tfs::kPbEta;
  dest_b[3 * m + 2] = sb + tfs::kPbS;
  dest_b[3 * m + 3] = sb + tfs::kPbInvDe;
  dest_b[3 * m + 4] = sb + tfs::kPbQ;
  dest_b[3 * m + 5] = -2;  // zeta of this step
  dest_b[3 * m + 6] = sb + tfs::kPbEtaRate;
  dest_b[3 * m + 7] = sb + tfs::kPbRate;
  dest_s[3 * m + 0] = sb + tfs::kPbInvDe;
  dest_s[3 * m + 1] = sb + tfs::kPbHgt;
  dest_s[3 * m + 2] = sb + tfs::kPbSrc1;
  dest_s[3 * m + 3] = sb + tfs::kPbSigma1;
  dest_s[3 * m + 4] = sb + tfs::kPbSigma2;
  dest_s[3 * m + 5] = sb + tfs::kPbGamma;
  dest_s[3 * m + 6] = sb + tfs::kPbTheta;
  dest_s[3 * m + 7] = sb + tfs::kPbHr;
  dest_s[3 * m + 8] = sb + tfs::kPbRate;
  // exponential-mode scheme: rows [0, m) dL/dw_k, [m, 2m) dL/dlambda_k, [2m, 3m) unused
  std::vector<int> dest_e(np, -1);
  for (int j = 0; j < 2 * m; ++j) dest_e[j] = j;
  dest_e[3 * m + 0] = sb + tfs::kPeA;
  dest_e[3 * m + 1] = sb + tfs::kPeQ;
  dest_e[3 * m + 2] = sb + tfs::kPeSh;
  dest_e[3 * m + 3] = sb + tfs::kPeInvDe;
  dest_e[3 * m + 4] = sb + tfs::kPeEtaE;
  dest_e[3 * m + 5] = -2;  // zeta of this step
  dest_e[3 * m + 6] = sb + tfs::kPeTs;
  dest_e[3 * m + 7] = sb + tfs::kPeQRate;
  dest_e[3 * m + 8] = sb + tfs::kPbRate;    // the rate gradient sits where the BDF2 scheme keeps it
  bool ok = hipMalloc(&p->d_adj_part, sizeof(double) * np * (size_t)std::max(1, p->part_cap)) == hipSuccess;
  ok = ok && hipMalloc(&p->d_dest_bdf2, sizeof(int) * np) == hipSuccess;
  ok = ok && hipMalloc(&p->d_dest_start, sizeof(int) * np) == hipSuccess;
  ok = ok && hipMalloc(&p->d_dest_exp, sizeof(int) * np) == hipSuccess;
  ok = ok && hipMemcpy(p->d_dest_exp, dest_e.data(), sizeof(int) * np, hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(p->d_dest_bdf2, dest_b.data(), sizeof(int) * np, hipMemcpyHostToDevice) == hipSuccess;
  ok = ok && hipMemcpy(p->d_dest_start, dest_s.data(), sizeof(int) * np, hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    (void)hipFree(p->d_coef); (void)hipFree(p->d_part); (void)hipFree(p->d_adj_part);
    (void)hipFree(p->d_dest_bdf2); (void)hipFree(p->d_dest_start); (void)hipFree(p->d_dest_exp);
    delete p;
    return fail(TFS_ENOMEM, "adjoint scratch");
  }
  *out = p;
  return TFS_OK;
}

tfs_status tfs_plan_destroy(tfs_plan p) {
  if (!p) return TFS_OK;
  hipError_t e1 = hipStreamSynchronize(p->stream);
  hipError_t e2 = hipFree(p->d_coef);
  hipError_t e3 = hipFree(p->d_part);
  (void)hipFree(p->d_adj_part);
  (void)hipFree(p->d_dest_bdf2);
  (void)hipFree(p->d_dest_start);
  (void)hipFree(p->d_dest_exp);
  (void)hipFree(p->d_field);
  (void)hipFree(p->d_field_roots);
  (void)hipFree(p->d_field_k);
  (void)hipFree(p->d_zeta);
  delete p;
  if (e1 != hipSuccess) return hip_fail(e1, "hipStreamSynchronize");
  if (e2 != hipSuccess) return hip_fail(e2, "hipFree");
  if (e3 != hipSuccess) return hip_fail(e3, "hipFree");
  return TFS_OK;
}

tfs_status tfs_plan_set_stream(tfs_plan p, void* stream) {
  if (!p) return fail(TFS_EINVAL, "null plan");
  p->stream = static_cast<hipStream_t>(stream);
  return TFS_OK;
}

tfs_status tfs_plan_set_field(tfs_plan p, const tfs_field* f) {
  if (!p || !f) return fail(TFS_EINVAL, "null plan or field");
  if (f->nterms < 0 || f->nterms > TFS_FIELD_MAX_TERMS)
    return fail(TFS_EINVAL, "nterms %d outside [0, %d]", f->nterms, TFS_FIELD_MAX_TERMS);
  if (f->grid < 1) return fail(TFS_EINVAL, "grid must be positive");
  int64_t cells = 1;
  for (int j = 0; j < p->d; ++j) {
    if (cells > std::numeric_limits<int64_t>::max() / f->grid) return fail(TFS_EINVAL, "grid^d overflows");
    cells *= f->grid;
  }
  if (f->point0 < 0 || f->point0 > cells - p->npoints)
    return fail(TFS_EINVAL, "points [point0, point0 + npoints) outside the grid");
  if (f->nterms > 0 && (!f->k || !f->phase || !f->omega || !f->coef))
    return fail(TFS_EINVAL, "null field table");
  const int d = p->d, W = d + 4 + d * d;
  std::vector<double> tab((size_t)std::max(1, f->nterms) * W, 0.0);
  bool steady = true;
  for (int n = 0; n < f->nterms; ++n) {
    double* r = tab.data() + (size_t)n * W;
    for (int j = 0; j < d; ++j) r[j] = f->k[n * d + j];
    r[d] = f->phase[n];
    r[d + 1] = f->omega[n];
    r[d + 2] = std::cos(f->omega[n] * p->dt);   // one step back by angle addition
    r[d + 3] = std::sin(f->omega[n] * p->dt);
    for (int q = 0; q < d * d; ++q) r[d + 4 + q] = f->coef[n * d * d + q];
    for (int q = 0; q < W; ++q)
      if (!std::isfinite(r[q])) return fail(TFS_EINVAL, "non-finite field table entry");
    if (f->omega[n] != 0.0) steady = false;
  }
  (void)hipSetDevice(p->device);
  double* dz = p->d_zeta;
  if (!dz) {
    hipError_t e = hipMalloc(&dz, sizeof(double) * p->zeta.size());
    if (e != hipSuccess) return fail(TFS_ENOMEM, "zeta table");
    e = hipMemcpy(dz, p->zeta.data(), sizeof(double) * p->zeta.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(dz); return hip_fail(e, "upload zeta"); }
    p->d_zeta = dz;
  }
  // the lattice form where every wave vector is an integer vector, |sum_j k_j idx_j| plus one
  // grid length stays in int32 (the evaluation's floor(m / grid) grid may sit a grid length
  // below m) and the roots of unity and the terms' rotations fit the evaluation's LDS
  bool lattice = f->nterms > 0 && 16 * (f->grid + (int64_t)f->nterms) <= tfs::kFieldLatticeLds;
  std::vector<int32_t> kint((size_t)std::max(1, f->nterms) * d, 0);
  for (int n = 0; lattice && n < f->nterms; ++n)
    for (int j = 0; j < d; ++j) {
      const double kv = f->k[n * d + j];
      if (kv != std::floor(kv) || (std::fabs(kv) * (double)d + 1.0) * (double)f->grid >= 2147483647.0)
        lattice = false;
      else kint[(size_t)n * d + j] = (int32_t)kv;
    }
  std::vector<double> roots(lattice ? (size_t)2 * f->grid : 0);
  for (int64_t m = 0; lattice && m < f->grid; ++m) {   // in extended precision, rounded once
    const long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)f->grid;
    roots[2 * m] = (double)std::cos(a);
    roots[2 * m + 1] = (double)std::sin(a);
  }
  double *df = nullptr, *dr = nullptr;
  int32_t* dk = nullptr;
  auto drop = [&]() {
    (void)hipFree(df);
    (void)hipFree(dr);
    (void)hipFree(dk);
  };
  hipError_t e = hipMalloc(&df, sizeof(double) * tab.size());
  if (e == hipSuccess && lattice) e = hipMalloc(&dr, sizeof(double) * roots.size());
  if (e == hipSuccess && lattice) e = hipMalloc(&dk, sizeof(int32_t) * kint.size());
  if (e != hipSuccess) { drop(); return fail(TFS_ENOMEM, "field table"); }
  e = hipMemcpy(df, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && lattice) e = hipMemcpy(dr, roots.data(), sizeof(double) * roots.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && lattice) e = hipMemcpy(dk, kint.data(), sizeof(int32_t) * kint.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) { drop(); return hip_fail(e, "upload field"); }
  e = hipStreamSynchronize(p->stream);   // launches that read the old tables have finished
  if (e != hipSuccess) { drop(); return hip_fail(e, "hipStreamSynchronize"); }
  (void)hipFree(p->d_field);
  (void)hipFree(p->d_field_roots);
  (void)hipFree(p->d_field_k);
  p->d_field = df;
  p->d_field_roots = dr;
  p->d_field_k = dk;
  p->field_terms = f->nterms;
  p->field_grid = f->grid;
  p->field_point0 = f->point0;
  p->field_steady = steady;
  return TFS_OK;
}

tfs_status tfs_run_fused(tfs_plan p, int64_t n0, int64_t nsteps, double* X, void* Y, double* tau) {
  if (!p) return fail(TFS_EINVAL, "null plan");
  if (!tfs::fused_supported(p))
    return fail(TFS_EUNSUPPORTED, "fused steps need m = 16 or 32, and FP32 modes in 3-D");
  if (p->zform) return fail(TFS_EUNSUPPORTED, "fused steps keep the modes in the Y form (TFS_MODE_FORM_Y)");
  if (p->scheme == TFS_SCHEME_BDF2 && n0 < 1 && nsteps > 0)
    return fail(TFS_EINVAL, "fused BDF2 steps start at level 1 or later (level 0 -> 1 is tfs_step's SDIRK2 start)");
  if (spatial(p)) return fail(TFS_EUNSUPPORTED, "no fused steps in the spatial form");
  if (!p->d_field) return fail(TFS_EINVAL, "no field set (tfs_plan_set_field)");
  if (n0 < 0 || nsteps < 0 || n0 > p->max_steps - nsteps)
    return fail(TFS_EINVAL, "levels [%lld, %lld] outside [0, %lld]", (long long)n0, (long long)(n0 + nsteps),
                (long long)p->max_steps);
  if (p->npoints > 0 && nsteps > 0 && (!X || !Y)) return fail(TFS_EINVAL, "null X or Y");
  hipError_t e = tfs::launch_fused(p, n0, nsteps, X, Y, tau);
  if (e != hipSuccess) return hip_fail(e, "fused launch");
  return TFS_OK;
}

tfs_status tfs_field_eval(tfs_plan p, double t, const double* add, void* kappa_out) {
  if (!p) return fail(TFS_EINVAL, "null plan");
  if (!p->d_field) return fail(TFS_EINVAL, "no field set (tfs_plan_set_field)");
  if (!std::isfinite(t)) return fail(TFS_EINVAL, "non-finite time");
  if (p->npoints > 0 && !kappa_out) return fail(TFS_EINVAL, "null kappa_out");
  hipError_t e = tfs::launch_field_eval(p, t, add, kappa_out);
  if (e != hipSuccess) return hip_fail(e, "field evaluation launch");
  return TFS_OK;
}

tfs_status tfs_plan_set_spatial(tfs_plan p, const double* rate, int64_t source_point) {
  if (!p) return fail(TFS_EINVAL, "null plan");
  if (source_point < -1 || source_point >= p->npoints)
    return fail(TFS_EINVAL, "source_point %lld outside [-1, npoints)", (long long)source_point);
  if (p->kappa_f32 && (rate || source_point >= 0))
    return fail(TFS_EUNSUPPORTED, "the spatial form takes FP64 velocity gradients");
  p->sp_rate = rate;
  p->sp_source = source_point;
  return TFS_OK;
}

int64_t tfs_plan_stride(tfs_plan p) { return p ? p->stride : -1; }

int64_t tfs_plan_tile(tfs_plan p) { return p ? (p->tile == p->stride ? 0 : p->tile) : -1; }

tfs_status tfs_plan_tune(tfs_plan p, const char* key, int64_t value) {
  if (!p || !key) return fail(TFS_EINVAL, "null plan or key");
  if (std::strcmp(key, "vec") == 0) {
    const bool ok = value == 0 || value == 1 || value == 2 || (value == 4 && p->precision == TFS_FP32_MODES);
    if (!ok) return fail(TFS_EINVAL, "vec must be 0, 1, 2 (or 4 for FP32 modes)");
    p->vec_override = (int)value;
    return TFS_OK;
  }
  if (std::strcmp(key, "adj_vec") == 0) {
    if (value < 0 || value > 2) return fail(TFS_EINVAL, "adj_vec must be 0, 1 or 2");
    p->adj_vec_override = (int)value;
    return TFS_OK;
  }
  if (std::strcmp(key, "grid_per_cu") == 0) {
    if (value < 1 || value > tfs::kMaxBlocksPerCU) return fail(TFS_EINVAL, "grid_per_cu must be in [1, 64]");
    p->grid_per_cu = (int)value;
    return TFS_OK;
  }
  return fail(TFS_EINVAL, "unknown tuning key '%s'", key);
}

tfs_status tfs_plan_tables(tfs_plan p, double* tables, double* scalars, double* zeta) {
  if (!p) return fail(TFS_EINVAL, "null plan");
  const int m = p->m;
  if (tables) {
    const int rows_b[5] = {tfs::kRowD, tfs::kRowC, tfs::kRowEta, tfs::kRowU, tfs::kRowV};
    const int rows_e[5] = {tfs::kRowE, tfs::kRowQ, tfs::kRowLdt, tfs::kRowOneME, tfs::kRowR};
    const int* rows = p->scheme == TFS_SCHEME_EXP ? rows_e : rows_b;
    for (int r = 0; r < 5; ++r)
      for (int k = 0; k < m; ++k) tables[r * m + k] = p->coef[rows[r] * m + k];
  }
  if (scalars) {
    const double v[8] = {p->eta, p->s_ec, p->a_diag, p->tau_scale, p->theta, p->rho, p->sigma1, p->sigma2};
    const double ve[8] = {p->q_e, p->s_h, p->a_diag, p->tau_scale, p->eta_e, 0.0, 0.0, 0.0};
    for (int i = 0; i < 8; ++i) scalars[i] = p->scheme == TFS_SCHEME_EXP ? ve[i] : v[i];
  }
  if (zeta) for (size_t i = 0; i < p->zeta.size(); ++i) zeta[i] = p->zeta[i];
  return TFS_OK;
}

namespace {

// Host chain rule of the exponential-mode scheme: the device already summed dL/dw_k and
// dL/dlambda_k through e_k, f_k, om_k, l_k (and q_k at level 0); what remains goes through
// the plan's scalars a = 1 + q/De, q = sum q_k, s_h = sum (om_k q_k - r_k),
// eta_e = dt sum (w_k - lambda_k q_k), ts = eta_p/(De dt), and the mass increments zeta.
// dL/dalpha = sum_k (dL/dw_k dw_k/dalpha + dL/dlambda_k dlambda_k/dalpha), Neumaier-compensated.
double alpha_chain(const std::vector<double>& wb, const std::vector<double>& lb, const double* dwa,
                   const double* dla) {
  double s = 0.0, comp = 0.0;
  auto add = [&](double x) {
    const double t = s + x;
    comp += std::fabs(s) >= std::fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
  };
  for (size_t k = 0; k < wb.size(); ++k) {
    add(wb[k] * dwa[k]);
    add(lb[k] * dla[k]);
  }
  return s + comp;
}

tfs_status exp_pbar_to_params(tfs_plan p, const double* pb, const double* dwa, const double* dla, double* dw,
                              double* dlam, double* dDe, double* deta_p, double* dalpha) {
  const int m = p->m;
  const double h = p->dt, iD = 1.0 / p->De;
  const double* sc = pb + 6 * m;
  const double* zb = pb + 6 * m + tfs::kPbarScalars;
  std::vector<double> wb(m), lb(m);
  for (int k = 0; k < m; ++k) { wb[k] = pb[k]; lb[k] = pb[m + k]; }
  const double qb = sc[tfs::kPeQ] + sc[tfs::kPeA] * iD + sc[tfs::kPeQRate];
  double iDb = sc[tfs::kPeInvDe] + sc[tfs::kPeA] * p->q_e;
  const double shb = sc[tfs::kPeSh], eeb = sc[tfs::kPeEtaE], tsb = sc[tfs::kPeTs];
  const int64_t N = p->max_steps;
  for (int k = 0; k < m; ++k) {
    const double wk = p->w[k], lk = p->lam[k];
    double e, om, a0, a1, b2;
    exp_mode_weights(lk * h, &e, &om, &a0, &a1, &b2);
    const double qk = wk * h * a1;
    const double dq_dw = h * a1, dq_dl = -wk * h * h * (a0 - b2);
    const double dr_dw = h * a0, dr_dl = -wk * h * h * b2;
    wb[k] += qb * dq_dw + shb * (om * dq_dw - dr_dw) + eeb * h * (1.0 - lk * dq_dw);
    lb[k] += qb * dq_dl + shb * (h * e * qk + om * dq_dl - dr_dl) - eeb * h * (qk + lk * dq_dl);
    // mass modes: mu^{n+1} = e mu^n + g, g = w dt (a0 + a1), zeta^{n+1} = sum_k (mu^{n+1} - mu^n)
    const double g = wk * h * (a0 + a1);
    std::vector<double> mu((size_t)N + 1, 0.0);
    for (int64_t n = 0; n < N; ++n) mu[n + 1] = e * mu[n] + g;
    double mub = 0.0, eb = 0.0, gb = 0.0;
    for (int64_t n = N - 1; n >= 0; --n) {
      mub += zb[n + 1];            // d zeta^{n+1} / d mu^{n+1}
      eb += mub * mu[n];
      gb += mub;
      mub = e * mub - zb[n + 1];   // to mu^n: through the recurrence and - mu^n in zeta^{n+1}
    }
    wb[k] += gb * h * (a0 + a1);
    lb[k] += -h * e * eb - gb * wk * h * h * a0;   // d(a0 + a1)/dz = -a0
  }
  // ts = eta_p / (De dt), 1/De
  const double eta_pb = tsb / (p->De * h);
  iDb += tsb * p->eta_p / h;
  if (dw) for (int k = 0; k < m; ++k) dw[k] = wb[k];
  if (dlam) for (int k = 0; k < m; ++k) dlam[k] = lb[k];
  if (dDe) *dDe = -iDb * iD * iD;
  if (deta_p) *deta_p = eta_pb;
  if (dalpha) *dalpha = alpha_chain(wb, lb, dwa, dla);
  return TFS_OK;
}

tfs_status run_step(tfs_plan p, int64_t n, const void* kappa_a, const void* kappa_b, const tfs::Levels& L,
                    double* tau, double* diag) {
  hipError_t e = p->scheme == TFS_SCHEME_EXP ? tfs::launch_exp(p, n, kappa_a, kappa_b, L, tau, diag)
                 : (n == 0) ? tfs::launch_startup(p, kappa_a, L, tau, diag)
                            : tfs::launch_bdf2(p, n, kappa_a, kappa_b, L, tau, diag);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  if (p->flags & TFS_FLAG_CHECK_SYNC) {
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    if (diag) {
      double h[tfs::kNumDiag];
      e = hipMemcpy(h, diag, sizeof(h), hipMemcpyDeviceToHost);
      if (e != hipSuccess) return hip_fail(e, "diagnostic read-back");
      if (h[5] != 0.0) return fail(TFS_ENUMERIC, "%g non-finite entries at level %lld", h[5], (long long)(n + 1));
      if (p->npoints > 0 && !spatial(p) && !(h[0] > 0.0 && h[1] > 0.0 && h[2] > 0.0))
        return fail(TFS_ENUMERIC, "conformation not positive definite at level %lld", (long long)(n + 1));
    }
  }
  return TFS_OK;
}

}  // namespace

namespace {

// tfs_step with the diagnostics block partials in `part` (null: the plan's buffer).
tfs_status step_ring(tfs_plan p, int64_t n, const void* kappa_a, const void* kappa_b, double* X, void* Y,
                     double* tau, double* diag, double* part) {
  if (!p) return fail(TFS_EINVAL, "null plan");
  if (n < 0 || n >= p->max_steps) return fail(TFS_EINVAL, "time level n=%lld outside [0, %lld)",
                                              (long long)n, (long long)p->max_steps);
  if (p->npoints > 0 && (!kappa_a || !X || !Y)) return fail(TFS_EINVAL, "null kappa_a, X or Y");
  const int64_t xs = (int64_t)p->c * p->stride, ys = (int64_t)p->m * p->c * p->stride;
  const size_t eb = p->precision == TFS_FP64 ? 8 : 4;
  char* Yb = static_cast<char*>(Y);
  tfs::Levels L;
  L.part = part;
  const int sn = (int)(n % 2), sm = 1 - sn;
  if (p->zform) {
    // three X levels; the mode ring as in the plain form
    const int64_t XL = p->xlev;
    if (n == 0) {
      L.Xn = X;
      L.Xo = X + xs;
      L.Ym0 = Yb;
      L.Yo = Yb + ys * eb;
    } else {
      L.Xn = X + (n % XL) * xs;
      L.Xm = X + ((n - 1) % XL) * xs;
      L.Xmm = n >= 2 ? X + ((n - 2) % XL) * xs : nullptr;
      L.Xo = X + ((n + 1) % XL) * xs;
      L.Yn = Yb + sn * ys * eb;
      L.Ym = Yb + sm * ys * eb;
      L.Yo = Yb + sm * ys * eb;
    }
    return run_step(p, n, kappa_a, kappa_b, L, tau, diag);
  }
  if (p->scheme == TFS_SCHEME_EXP) {
    L.Xn = X + sn * xs;
    L.Xo = X + sm * xs;
    L.Yn = Yb;
    L.Yo = Yb;
    return run_step(p, n, kappa_a, kappa_b, L, tau, diag);
  }
  if (n == 0) {
    L.Xn = X;
    L.Xo = X + xs;
    L.Ym0 = Yb;
    L.Yo = Yb + ys * eb;
  } else {
    L.Xn = X + sn * xs;
    L.Xm = X + sm * xs;
    L.Xo = X + sm * xs;
    L.Yn = Yb + sn * ys * eb;
    L.Ym = Yb + sm * ys * eb;
    L.Yo = Yb + sm * ys * eb;
  }
  return run_step(p, n, kappa_a, kappa_b, L, tau, diag);
}

}  // namespace

tfs_status tfs_step(tfs_plan p, int64_t n, const void* kappa_a, const void* kappa_b, double* X, void* Y,
                    double* tau, double* diag) {
  return step_ring(p, n, kappa_a, kappa_b, X, Y, tau, diag, nullptr);
}

tfs_status tfs_step_noalloc(tfs_plan p, int64_t n, const void* kappa_a, const void* kappa_b, double* X, void* Y,
                            double* tau, double* diag) {
  if (!p) return fail(TFS_EINVAL, "null plan");
  if (!diag) return step_ring(p, n, kappa_a, kappa_b, X, Y, tau, nullptr, nullptr);
  if (!p->d_scratch)
    return fail(TFS_EHIP, "static scratch unavailable on device %d: %s", p->device,
                hipGetErrorString((hipError_t)p->scratch_err));
  // a V-wide pass and a tail pass, each of at most num_cus * grid_per_cu blocks
  const int64_t need = 2 * (int64_t)p->num_cus * p->grid_per_cu;
  if (need > tfs::kScratchPartials)
    return fail(TFS_EINVAL,
                "the step's launches write up to %lld diagnostics partials (2 x %d CUs x grid_per_cu %d); the "
                "static scratch holds %d: lower grid_per_cu (tfs_plan_tune)",
                (long long)need, p->num_cus, p->grid_per_cu, tfs::kScratchPartials);
  return step_ring(p, n, kappa_a, kappa_b, X, Y, tau, diag, p->d_scratch);
}

tfs_status tfs_step_levels(tfs_plan p, int64_t n, const void* kappa_a, const void* kappa_b, const double* X_n,
                           const double* X_nm1, const double* X_nm2, double* X_out, const void* Y_n, void* Y_nm1,
                           void* Y_out, double* tau, double* diag) {
  if (!p) return fail(TFS_EINVAL, "null plan");
  if (n < 0 || n >= p->max_steps) return fail(TFS_EINVAL, "time level n=%lld outside [0, %lld)",
                                              (long long)n, (long long)p->max_steps);
  if (p->scheme == TFS_SCHEME_EXP) {
    if (p->npoints > 0) {
      if (!kappa_a || !X_n || !X_out || !Y_out) return fail(TFS_EINVAL, "null kappa_a, X or Y level");
      if (n > 0 && !Y_n) return fail(TFS_EINVAL, "null Y_n");
      if (X_out == X_n) return fail(TFS_EINVAL, "X_out must not alias X_n");
    }
    tfs::Levels L;
    L.Xn = X_n;
    L.Xo = X_out;
    L.Yn = n > 0 ? Y_n : Y_out;
    L.Yo = Y_out;
    return run_step(p, n, kappa_a, kappa_b, L, tau, diag);
  }
  if (p->npoints > 0) {
    if (!kappa_a || !X_n || !X_out || !Y_nm1 || !Y_out) return fail(TFS_EINVAL, "null kappa_a, X or Y level");
    if (n > 0 && (!X_nm1 || !Y_n)) return fail(TFS_EINVAL, "null level n or n-1");
    if (p->zform && n > 1 && !X_nm2) return fail(TFS_EINVAL, "null level n-2 (shifted mode form)");
    if (X_out == X_n) return fail(TFS_EINVAL, "X_out must not alias X_n");
    if (n > 0 && Y_out == Y_n) return fail(TFS_EINVAL, "Y_out must not alias Y_n");
  }
  tfs::Levels L;
  L.Xn = X_n;
  L.Xo = X_out;
  if (n == 0) {
    L.Ym0 = Y_nm1;
    L.Yo = Y_out;
  } else {
    L.Xm = X_nm1;
    L.Xmm = (p->zform && n > 1) ? X_nm2 : nullptr;
    L.Yn = Y_n;
    L.Ym = Y_nm1;
    L.Yo = Y_out;
  }
  return run_step(p, n, kappa_a, kappa_b, L, tau, diag);
}

int64_t tfs_pbar_size(tfs_plan p) {
  return p ? 6 * (int64_t)p->m + tfs::kPbarScalars + p->max_steps + 1 : -1;
}

tfs_status tfs_pbar_rate_gradient(tfs_plan p, const double* pbar_host, double* out) {
  if (!p || !pbar_host || !out) return fail(TFS_EINVAL, "null plan, pbar or out");
  *out = pbar_host[6 * (int64_t)p->m + tfs::kPbRate];
  return TFS_OK;
}

tfs_status tfs_step_adjoint(tfs_plan p, int64_t n, const void* kappa_a, const void* kappa_b, const double* X_n,
                            const double* X_nm1, const double* X_nm2, const double* X_np1, const void* Y_n,
                            const void* Y_nm1,
                            double* Xbar, void* Hbar, const double* taubar, double* kappabar_a,
                            double* kappabar_b, double* pbar) {
  if (!p) return fail(TFS_EINVAL, "null plan");
  if (n < 0 || n >= p->max_steps) return fail(TFS_EINVAL, "time level n=%lld outside [0, %lld)",
                                              (long long)n, (long long)p->max_steps);
  if (!pbar) return fail(TFS_EINVAL, "null pbar");
  if (p->npoints > 0) {
    if (!kappa_a || !X_n || !Xbar || !Hbar) return fail(TFS_EINVAL, "null kappa_a, X_n, Xbar or Hbar");
    if (p->scheme == TFS_SCHEME_EXP) {
      if (!X_np1 || (n > 0 && !Y_n)) return fail(TFS_EINVAL, "null forward level");
    } else if (n > 0 && (!X_nm1 || !X_np1 || !Y_n || !Y_nm1)) {
      return fail(TFS_EINVAL, "null forward level");
    } else if (p->zform && n > 1 && !X_nm2) {
      return fail(TFS_EINVAL, "null forward level n-2 (shifted mode form)");
    }
  }
  tfs::AdjLevels L;
  L.ka = kappa_a;
  L.kb = n > 0 ? kappa_b : nullptr;
  L.Xn = X_n;
  L.Xm = X_nm1;
  L.Xmm = (p->zform && n > 1) ? X_nm2 : nullptr;
  L.Xp = X_np1;
  L.Yn = Y_n;
  L.Ym = Y_nm1;
  L.Xbar = Xbar;
  L.Hbar = Hbar;
  L.taubar = taubar;
  L.kba = kappabar_a;
  L.kbb = kappabar_b;
  hipError_t e = tfs::launch_adjoint(p, n, L, pbar);
  if (e != hipSuccess) return hip_fail(e, "adjoint launch");
  return TFS_OK;
}

tfs_status tfs_pbar_to_params(tfs_plan p, const double* pb, const double* dwa, const double* dla, double* dw,
                              double* dlam, double* dDe, double* deta_p, double* dalpha) {
  if (!p || !pb) return fail(TFS_EINVAL, "null plan or pbar");
  if (dalpha && (!dwa || !dla)) return fail(TFS_EINVAL, "dL/dalpha needs dw/dalpha and dlambda/dalpha");
  if (p->scheme == TFS_SCHEME_EXP) return exp_pbar_to_params(p, pb, dwa, dla, dw, dlam, dDe, deta_p, dalpha);
  const int m = p->m;
  const double h = p->dt, b0 = tfs::kB0, gs = 1.0 - 1.0 / std::sqrt(2.0), hg = h * gs, hs = h * (1.0 - gs);
  const double iD = 1.0 / p->De;
  const double* sc = pb + 6 * m;
  const double* zb = pb + 6 * m + tfs::kPbarScalars;
  std::vector<double> wb(m, 0.0), lb(m, 0.0), db(m, 0.0), cb(m, 0.0), ekb(m, 0.0);
  for (int k = 0; k < m; ++k) {
    db[k] = pb[k];
    ekb[k] = pb[2 * m + k];
    cb[k] = pb[3 * m + k];                // start-up Y^0 = -c X^0
  }
  // scalar chain: a = b0 + eta/De, q = gamma/dt, gamma = eta_p/De
  double etab = sc[tfs::kPbEta] + sc[tfs::kPbA] * iD + sc[tfs::kPbEtaRate];
  double iDb = sc[tfs::kPbInvDe] + sc[tfs::kPbA] * p->eta;
  const double gammab = sc[tfs::kPbGamma] + sc[tfs::kPbQ] / h;
  const double eta_pb = gammab * iD;
  iDb += gammab * p->eta_p;
  // start-up scalars
  double thetab = hg * (sc[tfs::kPbHgt] + sc[tfs::kPbSrc1]) + hs * sc[tfs::kPbSigma1] + h * sc[tfs::kPbSigma2] +
                  sc[tfs::kPbTheta];
  double rhob = -hs * hg * sc[tfs::kPbSigma1] - hg * hs * sc[tfs::kPbSigma2] + hs * sc[tfs::kPbHr];
  // mass-mode memory: reverse the mu recurrence driving zeta
  {
    const int64_t N = p->max_steps;
    std::vector<double> mu((size_t)(N + 1) * m, 0.0);
    for (int k = 0; k < m; ++k) {
      const double r = 1.0 / (1.0 + hg * p->lam[k]);
      mu[(size_t)1 * m + k] = (hs * p->w[k] * r + hg * p->w[k]) * r;
    }
    for (int64_t n = 1; n < N; ++n)
      for (int k = 0; k < m; ++k) {
        const double hh = 2.0 * mu[(size_t)n * m + k] - 0.5 * mu[(size_t)(n - 1) * m + k];
        mu[(size_t)(n + 1) * m + k] = p->coef[tfs::kRowD * m + k] * hh + p->coef[tfs::kRowC * m + k];
      }
    std::vector<double> mub((size_t)(N + 1) * m, 0.0);
    for (int64_t n = N - 1; n >= 1; --n) {
      const double zbar = zb[n + 1];
      etab += zbar;
      for (int k = 0; k < m; ++k) {
        const double hh = 2.0 * mu[(size_t)n * m + k] - 0.5 * mu[(size_t)(n - 1) * m + k];
        const double mup = mub[(size_t)(n + 1) * m + k];
        db[k] += mup * hh;
        cb[k] += mup;
        ekb[k] += -zbar * hh;
        const double hb = p->coef[tfs::kRowD * m + k] * mup - zbar * p->coef[tfs::kRowEta * m + k];
        mub[(size_t)n * m + k] += 2.0 * hb;
        mub[(size_t)(n - 1) * m + k] += -0.5 * hb;
      }
    }
    for (int k = 0; k < m; ++k) {
      const double w = p->w[k], r = 1.0 / (1.0 + hg * p->lam[k]);
      const double g = mub[(size_t)1 * m + k];
      wb[k] += g * (hs * r * r + hg * r);
      lb[k] += g * (-2.0 * hs * hg * w * r * r * r - hg * hg * w * r * r);
    }
  }
  // per-mode start-up factors theta, rho, u_k, v_k
  for (int k = 0; k < m; ++k) {
    const double w = p->w[k], l = p->lam[k], r = 1.0 / (1.0 + hg * l);
    wb[k] += thetab * r;
    lb[k] += thetab * w * (-hg * r * r);
    wb[k] += rhob * l * r * r;
    lb[k] += rhob * w * r * r * (1.0 - 2.0 * hg * l * r);
    const double ub = pb[4 * m + k], vb = pb[5 * m + k];
    wb[k] += ub * hs * r * r;
    lb[k] += -2.0 * ub * hs * hg * w * r * r * r;
    wb[k] += vb * hg * r;
    lb[k] += vb * hg * w * (-hg * r * r);
    cb[k] += -vb;
  }
  // BDF2 factors: eta = sum b0 c_k, s = sum eta_k c_k, e_k = d_k c_k, c_k = w dt d_k,
  // eta_k = lambda dt d_k, d_k = 1/(b0 + lambda dt)
  const double sb = sc[tfs::kPbS];
  for (int k = 0; k < m; ++k) {
    const double w = p->w[k], l = p->lam[k];
    const double d = p->coef[tfs::kRowD * m + k], c = p->coef[tfs::kRowC * m + k];
    const double ek = p->coef[tfs::kRowEta * m + k];
    double ck = cb[k] + b0 * etab + sb * ek;
    double ekk = ekb[k] + sb * c;
    const double eb = pb[m + k];             // d(Y)/d(d_k c_k)
    double dk = db[k] + eb * c;
    ck += eb * d;
    wb[k] += ck * h * d;
    dk += ck * w * h;
    lb[k] += ekk * h * d;
    dk += ekk * l * h;
    lb[k] += dk * (-h * d * d);
  }
  if (dw) for (int k = 0; k < m; ++k) dw[k] = wb[k];
  if (dlam) for (int k = 0; k < m; ++k) dlam[k] = lb[k];
  if (dDe) *dDe = -iDb * iD * iD;
  if (deta_p) *deta_p = eta_pb;
  if (dalpha) *dalpha = alpha_chain(wb, lb, dwa, dla);
  return TFS_OK;
}

tfs_status tfs_modes_to_plain(tfs_plan p, int64_t level, const double* X, const void* Y, double* Xk_out) {
  if (!p) return fail(TFS_EINVAL, "null plan");
  if (level < 0) return fail(TFS_EINVAL, "level must be >= 0");
  if (p->npoints > 0 && (!X || !Y || !Xk_out)) return fail(TFS_EINVAL, "null pointer");
  hipError_t e = tfs::launch_modes_to_plain(p, level, X, Y, Xk_out);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return TFS_OK;
}

int32_t tfs_plan_x_levels(tfs_plan p) { return p ? p->xlev : -1; }

}  // extern "C"

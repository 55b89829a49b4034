// Internal definitions shared by the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "tfs.h"

namespace tfs {

// BDF2 coefficients b_0, b_1, b_2 and the SDIRK2 diagonal (Alexander's L-stable
// two-stage method, first step only).
constexpr double kB0 = 1.5;
constexpr double kB1 = -2.0;
constexpr double kB2 = 0.5;

// Rows of the device coefficient table [kNumCoef][m].
enum CoefRow : int {
  kRowD = 0,    // d_k = 1/(b0 + lambda_k dt)
  kRowDC = 1,   // d_k c_k
  kRowEta = 2,  // eta_k = lambda_k dt d_k
  kRowC = 3,    // c_k = w_k dt d_k
  kRowU = 4,    // start-up: coefficient of the first stage value in Y_k^1
  kRowV = 5,    // start-up: coefficient of the second stage value in Y_k^1
  kRowBeta = 6, // shifted mode form: beta_k = w_k/lambda_k - c_k (0 for lambda_k = 0 or the plain form)
  kNumCoef = 7
};

// Rows of the same table for TFS_SCHEME_EXP plans (exponential mode update).
enum ExpRow : int {
  kRowE = 0,      // e_k = exp(-lambda_k dt)
  kRowF = 1,      // f_k = e_k q_k + w_k dt a0_k: coefficient of X^n in Y_k^{n+1}
  kRowLdt = 2,    // lambda_k dt
  kRowQ = 3,      // q_k = w_k dt a1_k (plain modes X_k = Y_k + q_k X; same row as c_k)
  kRowOneME = 4,  // 1 - e_k
  kRowR = 5,      // w_k dt a0_k
  // adjoint: derivatives of the step's per-mode factors (w_k, lambda_k chain on the device)
  kRowFW = 6,     // d f_k / d w_k
  kRowFL = 7,     // d f_k / d lambda_k
  kRowQW = 8,     // -d q_k / d w_k       (level 0: Y_k^0 = -q_k X^0)
  kRowQL = 9      // -d q_k / d lambda_k
};
constexpr int kNumCoefAll = 10;   // rows of the table (BDF2 plans use the first kNumCoef)

// Scalar positions in pbar for TFS_SCHEME_EXP plans (after the 6 m per-mode entries, of
// which [0, m) hold dL/dw_k and [m, 2m) dL/dlambda_k from the device).
enum PbarExpScalar : int { kPeA = 0, kPeQ = 1, kPeSh = 2, kPeInvDe = 3, kPeEtaE = 4, kPeTs = 5,
                           kPeQRate = 6 };   // spatial form: sum_p rate_p dL/da_p (adds to dL/dq)

// Number of diagnostics written per step.
constexpr int kNumDiag = 6;
// Largest number of sum-of-exponentials modes of a plan (bounds the adjoint LDS use).
constexpr int kMaxModes = 256;
// Threads per block of every streaming kernel.
constexpr int kBlock = 256;
// Upper bound of blocks per compute unit of the grid-stride launches (sizes the
// diagnostic scratch).
constexpr int kMaxBlocksPerCU = 64;
// LDS (bytes) of the field evaluation's lattice form: the grid's roots of unity and one
// rotation per term, 16 bytes each
constexpr int64_t kFieldLatticeLds = 32768;
// Scalar sums per block of one adjoint launch, and the scalar block of pbar.
constexpr int kNumAdjScalars = 9;
constexpr int kPbarScalars = 16;
// Scalar positions in pbar (after the 6 m per-mode entries).
enum PbarScalar : int {
  kPbA = 0, kPbEta = 1, kPbS = 2, kPbInvDe = 3, kPbQ = 4, kPbHgt = 5, kPbSrc1 = 6, kPbSigma1 = 7,
  kPbSigma2 = 8, kPbGamma = 9, kPbTheta = 10, kPbHr = 11,
  // spatial form: sum_p rate_p dL/da_p (adds to dL/deta) and sum_p rate_p dL/drate_p
  kPbEtaRate = 12, kPbRate = 13
};

// Per-step scalars of the BDF2 update, all FP64.
struct Bdf2Scalars {
  double a_diag;     // b0 + eta/De: diagonal of the local operator
  double eta;        // eta = sum_k b0 c_k
  double s_ec;       // sum_k eta_k c_k
  double inv_De;     // 1/De
  double zeta;       // mass-mode memory term zeta^{n+1}
  double tau_scale;  // gamma/dt
};

// Per-step scalars of the exponential-mode step (TFS_SCHEME_EXP), all FP64.
struct ExpScalars {
  double a_diag;     // 1 + q/De: diagonal of the local operator
  double q;          // q = sum_k q_k: weight of K X^{n+1}
  double s_h;        // sum_k ((1 - e_k) q_k - w_k dt a0_k): X^n part of the mode decrement H
  double inv_De;
  double zeta;       // sum_k (mu_k^{n+1} - mu_k^n): the mass modes' increment
  double tau_scale;  // gamma/dt
  double eta_e;      // dt sum_k (w_k - lambda_k q_k): dt D^{1-alpha} X^{n+1} = eta_e X^{n+1} - G
  double fa, fb;     // kappa~ = fa kappa_a + fb kappa_b
  int first;         // n = 0: Y^0 = -q_k X^0, the mode input is not read
};

// Scalars of the SDIRK2 start-up step.
struct StartScalars {
  double hgt;        // h gs theta: off-identity weight of the stage matrix
  double inv_De;
  double src1;       // h gs theta: source weight of stage 1
  double sigma1;     // weight of A(X^(1)) in stage 2
  double sigma2;     // weight of S in stage 2
  double gamma;      // eta_p/De
  double theta;
  double hr;         // h (1 - gs) rho
};

}  // namespace tfs

struct tfs_plan_s {
  int d = 0, c = 0, m = 0;
  int64_t npoints = 0, stride = 0, max_steps = 0;
  int64_t tile = 0;           // mode-ring tile (points); equals stride when untiled
  double alpha = 0, De = 0, eta_p = 0, dt = 0, gamma = 0;
  int precision = 0;
  bool kappa_f32 = false;     // velocity gradients stored in FP32 (FP32-mode plans only)
  // BDF2 mode representation: Y-form Y_k^j = X_k^j - c_k X^j, or the shifted form
  // Z_k^j = Y_k^j - beta_k X^{j-1} (X^{-1} = 0), which needs X at three levels
  bool zform = false;
  int xlev = 2;               // slots of the X ring (3 with the shifted form)
  int scheme = TFS_SCHEME_BDF2;
  uint32_t flags = 0;
  hipStream_t stream = nullptr;
  int device = 0;

  std::vector<double> w, lam;
  std::vector<double> coef;   // host copy of [kNumCoefAll][m]
  double eta = 0, s_ec = 0, a_diag = 0, tau_scale = 0;
  double theta = 0, rho = 0, sigma1 = 0, sigma2 = 0, hg = 0, hr = 0;
  double q_e = 0, s_h = 0, eta_e = 0;   // TFS_SCHEME_EXP scalars (ExpScalars)
  std::vector<double> zeta;   // [max_steps + 1]

  double* d_coef = nullptr;   // device [kNumCoefAll][m]
  double* d_part = nullptr;   // device [part_cap][kNumDiag] block partials
  int part_cap = 0;
  double* d_adj_part = nullptr;  // device [part_cap][3 m + kNumAdjScalars] adjoint block partials
  int* d_dest_bdf2 = nullptr;    // device [3 m + kNumAdjScalars]: pbar index of each partial entry
  int* d_dest_start = nullptr;
  int* d_dest_exp = nullptr;
  // the calling device's static scratch (tfs_step_noalloc), looked up at plan creation
  double* d_scratch = nullptr;
  int scratch_err = 0;        // hipError_t of that lookup

  // tuning (tfs_plan_tune): points per lane (0 = widest aligned), blocks per CU cap
  int vec_override = 0;
  int adj_vec_override = 0;
  // analytic velocity-gradient field of the fused launches (tfs_plan_set_field)
  double* d_field = nullptr;         // device [field_terms][d + 2 + d*d]
  double* d_zeta = nullptr;          // device copy of zeta
  int field_terms = 0;
  int64_t field_grid = 0, field_point0 = 0;
  bool field_steady = false;
  // lattice form of the field (integer wave vectors, small grid): the grid's roots of unity
  // (cos, sin)(2 pi m / grid), m < grid, and the wave vectors as integers; null otherwise
  double* d_field_roots = nullptr;   // device [field_grid][2]
  int32_t* d_field_k = nullptr;      // device [field_terms][d]
  const double* sp_rate = nullptr;   // spatial form: extra relaxation rate per point (caller-owned)
  int64_t sp_source = -1;            // spatial form: the point with the mass-mode source, -1 = all
  int grid_per_cu = 16;
  int num_cus = 256;
  int lds_max = 65536;      // LDS bytes a block may use on the plan's device
};

namespace tfs {

// Time-level pointers of one step: BDF2 reads (Xn, Xm, Yn, Ym) and writes (Xo, Yo); the
// start-up reads Xn = X^0 and writes Xo = X^1, Ym0 = Y^0 and Yo = Y^1.
struct Levels {
  const double* Xn = nullptr;
  const double* Xm = nullptr;
  const double* Xmm = nullptr;  // X^{n-2} (shifted mode form, n >= 2; null: zero)
  double* Xo = nullptr;
  const void* Yn = nullptr;
  const void* Ym = nullptr;
  void* Ym0 = nullptr;
  void* Yo = nullptr;
  double* part = nullptr;       // block partials of the diagnostics (null: the plan's d_part)
};

// Pointers of one adjoint step.
struct AdjLevels {
  const void* ka = nullptr;     // plan's kappa precision
  const void* kb = nullptr;
  const double* Xn = nullptr;   // forward X^n (X^0 at n = 0)
  const double* Xm = nullptr;   // forward X^{n-1}
  const double* Xmm = nullptr;  // forward X^{n-2} (shifted mode form, n >= 2; null: zero)
  const double* Xp = nullptr;   // forward X^{n+1}
  const void* Yn = nullptr;     // forward Y^n
  const void* Ym = nullptr;     // forward Y^{n-1}
  double* Xbar = nullptr;       // adjoint ring [xlev][c][stride]
  void* Hbar = nullptr;         // mode-adjoint ring, 2 slots
  const double* taubar = nullptr;
  double* kba = nullptr;
  double* kbb = nullptr;
};

// Launchers (tfs_kernels.hip, tfs_adjoint.hip).  They only enqueue work on plan->stream.
hipError_t launch_adjoint(const tfs_plan_s* p, int64_t n, const AdjLevels& L, double* pbar);
// Fused exponential-mode steps with kappa from the plan's analytic field (tfs_fused.hip).
bool fused_supported(const tfs_plan_s* p);
hipError_t launch_fused(const tfs_plan_s* p, int64_t n0, int64_t nsteps, double* X, void* Y, double* tau);
// ka, kb: velocity gradients in the plan's kappa precision (FP64, or FP32 when kappa_f32).
hipError_t launch_bdf2(const tfs_plan_s* p, int64_t n, const void* ka, const void* kb, const Levels& L,
                       double* tau, double* diag);
hipError_t launch_startup(const tfs_plan_s* p, const void* ka, const Levels& L, double* tau, double* diag);
// BDF2 step n >= 1 without the local solve: writes Y^{n+1} (L.Yo), the right-hand side R of
// each point (L.Xo) and the history combination G ([c][stride]); no diagnostics.
hipError_t launch_bdf2_split(const tfs_plan_s* p, int64_t n, const double* ka, const double* kb, const Levels& L,
                             double* G);
// Exponential-mode step n -> n+1 (TFS_SCHEME_EXP): reads L.Xn and L.Yn (not at n = 0),
// writes L.Xo and L.Yo (which may be L.Yn).
hipError_t launch_exp(const tfs_plan_s* p, int64_t n, const void* ka, const void* kb, const Levels& L,
                      double* tau, double* diag);
// Exponential-mode step without the local solve: writes Y^{n+1} (L.Yo, may be L.Yn), the
// right-hand side R of each point (L.Xo), G and H ([c][stride] each); no diagnostics.
hipError_t launch_exp_split(const tfs_plan_s* p, int64_t n, const double* ka, const double* kb, const Levels& L,
                            double* G, double* H);
hipError_t launch_modes_to_plain(const tfs_plan_s* p, int64_t level, const double* X, const void* Y,
                                 double* Xk);
// kappa_out [d*d][stride] (plan's kappa precision) = the plan's analytic field at time t, plus
// add [d*d][stride] FP64 when add is not null (tfs_field.hip).
hipError_t launch_field_eval(const tfs_plan_s* p, double t, const double* add, void* out);
// Upper bound of blocks the launchers use for a plan (sizes d_part).
int max_blocks(const tfs_plan_s* p);
// Block partials the static scratch holds (tfs_step_noalloc).
constexpr int kScratchPartials = 2 * 256 * 16;
// Device address of the static scratch on the current device, looked up once per device
// (tfs_kernels.hip).
hipError_t scratch_address(int device, double** out);

}  // namespace tfs

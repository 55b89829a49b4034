"""The oracle pins must catch plausible mistakes.

Each case plants one mistake in a copy of the oracle source (on the CPU, in a
temporary directory), builds it, and runs the pin tests against that library in
a subprocess; at least one pin must fail.  The real oracle is untouched.
"""
import os
import subprocess
import sys

import pytest

from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "tfs_oracle.c")

# name -> (original text, planted mistake, pytest -k expression of pins expected to fail[,
#          pin file; default test_oracle_pins.py])
MUTATIONS = {
    "transposed_kappa": ("const sc kml = kap[m * d + l];", "const sc kml = kap[l * d + m];", "operator"),
    "dropped_stretch_term": ("((2.0 * a * a - 1.0) / (2.0 * De) + kap[l * d + l])",
                             "((2.0 * a * a - 1.0) / (2.0 * De))", "operator"),
    "half_relaxation": ("diag += (kap[l * d + l] - 1.0 / (2.0 * De))",
                        "diag += (kap[l * d + l] - 1.0 / (4.0 * De))", "operator"),
    "bdf2_coefficient_sign": ("const double b0 = 1.5, b1 = -2.0, b2 = 0.5;",
                              "const double b0 = 1.5, b1 = -2.0, b2 = -0.5;", "alpha_one"),
    "eta_k_with_weight": ("const sc etak = lam[k] * dt / (b0 + lam[k] * dt);",
                          "const sc etak = w[k] * dt / (b0 + lam[k] * dt);", "brute_force"),
    "sdirk_diagonal": ("const rl gs = 1 - 1 / SQRTR((rl)2);", "const rl gs = 0.5;", "sdirk2 or alpha_one"),
    "recombination_sign": ("terms[k] = w[k] * Pnew[q] - lam[k] * Knew[k * n + q];",
                           "terms[k] = w[k] * Pnew[q] + lam[k] * Knew[k * n + q];", "brute_force or sdirk2"),
    "stage_two_explicit_part": ("E[q] = Pn[q] + dt * (1.0 - gs) * F1[q];", "E[q] = Pn[q];", "sdirk2"),
    "hermite_map_scale": ("else if (i1 == i2) Phi[r] = Xfull[i1 * d + i1] / SQRTR((rl)2);",
                          "else if (i1 == i2) Phi[r] = Xfull[i1 * d + i1] / 2.0;", "hermite_map or operator"),
    "mode_push_dropped_level": ("Km[k * n + q] = (-(b1 * Kn[k * n + q] + b2 * Km[k * n + q]) + w[k] * dt * rhs[q]) /",
                                "Km[k * n + q] = (-(b1 * Kn[k * n + q]) + w[k] * dt * rhs[q]) /", "brute_force"),
    "eta_without_b0": ("eta += b0 * w[k] * dt / (b0 + lam[k] * dt);", "eta += w[k] * dt / (b0 + lam[k] * dt);",
                       "alpha_one or brute_force"),
    "no_extrapolation": ("kt[q] = fa * ka[q] + fb * kb[q];", "kt[q] = ka[q];", "time_varying"),
    "mass_switch_ignored": ("tensor_to_hermite(&h, Xf, mass ? (sc)mass[p] : (sc)1.0, P0);",
                            "tensor_to_hermite(&h, Xf, (sc)1.0, P0);", "mass_free"),
    # exponential-mode scheme (pins in test_oracle_exp_pins.py)
    "exp_weights_swapped": ("Km[k * n + i] = e * Kn[k * n + i] + w[k] * dt * (a0 * Pn[i] + a1 * rhs[i]);",
                            "Km[k * n + i] = e * Kn[k * n + i] + w[k] * dt * (a1 * Pn[i] + a0 * rhs[i]);",
                            "relaxation or general_kappa", "test_oracle_exp_pins.py"),
    "exp_decrement_without_decay": ("v[i] += (e - 1.0) * Kn[k * n + i] + w[k] * dt * a0 * Pn[i];",
                                    "v[i] += -Kn[k * n + i] + w[k] * dt * a0 * Pn[i];",
                                    "relaxation or general_kappa", "test_oracle_exp_pins.py"),
    "exp_series_term": ("s1 += t / ((double)(j + 1) * (double)(j + 2));", "s1 += t / ((double)(j + 2) * (double)(j + 2));",
                        "weights", "test_oracle_exp_pins.py"),
    "exp_kappa_at_full_step": ("const double fa = startup == 2 ? 1.5 : 2.0, fb = startup == 2 ? -0.5 : -1.0;",
                               "const double fa = 2.0, fb = -1.0;", "time_varying", "test_oracle_exp_pins.py"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_fails_a_pin(name, tmp_path):
    orig, bad, sel = MUTATIONS[name][:3]
    pins = MUTATIONS[name][3] if len(MUTATIONS[name]) > 3 else "test_oracle_pins.py"
    src = open(SRC).read()
    assert src.count(orig) == 1, "mutation anchor drifted from the oracle source"
    msrc = tmp_path / "mutant.c"
    msrc.write_text(src.replace(orig, bad))
    lib = str(tmp_path / "libmutant.so")
    obuild.build(src=str(msrc), lib=lib)
    env = dict(os.environ, TFS_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", pins),
                        "-q", "-x", "-p", "no:cacheprovider", "-k", sel],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"no pin caught '{name}':\n{r.stdout[-2000:]}"


# Mistakes planted in the spatial oracle (oracle/mfp.py; pins in test_oracle_mfp_pins.py).
MFP_SRC = os.path.join(ROOT, "oracle", "mfp.py")
MFP_MUTATIONS = {
    "history_without_laplacian": ("rhs = -(B1 * phi[0] + B2 * phi[1]) + A @ hist",
                                  "rhs = -(B1 * phi[0] + B2 * phi[1]) + (A - eps * np.kron(lap, np.eye(n))) @ hist",
                                  "fourier_mode or convergence"),
    "laplacian_sign": ("A = eps * np.kron(lap, np.eye(n))", "A = -eps * np.kron(lap, np.eye(n))",
                       "fourier_mode or convergence"),
    "sdirk_stage_without_laplacian": ("F1 = A @ np.sum(Fk, axis=0)",
                                      "F1 = (A - eps * np.kron(lap, np.eye(n))) @ np.sum(Fk, axis=0)",
                                      "fourier_mode"),
    "nyquist_dropped": ("return sum(g * g for g in grids)",
                        "return sum(np.where(np.abs(g) >= np.max(np.abs(g)) - 1e-9, 0.0, g * g) for g in grids)",
                        "trigonometric"),
    "advection_sign": ("A -= np.kron(adv, np.eye(n))", "A += np.kron(adv, np.eye(n))", "complex_rate"),
    "exp_history_without_laplacian": ("new_phi = np.linalg.solve(I - q_exp * A, phi[0] + A @ v)",
                                      "new_phi = np.linalg.solve(I - q_exp * A, phi[0] + "
                                      "(A - eps * np.kron(lap, np.eye(n))) @ v)", "fourier_mode and exp"),
    "exp_half_step_as_bdf2": ("fa, fb = (2.0, -1.0) if scheme == \"bdf2\" else (1.5, -0.5)",
                              "fa, fb = (2.0, -1.0)", "pointwise_oracle and exp"),
    "derivative_on_the_wrong_axis": ("sym = k.reshape([n if j == axis else 1 for j in range(len(shape))])",
                                     "sym = k.reshape([n if j == len(shape) - 1 - axis else 1 "
                                     "for j in range(len(shape))]) if len(set(shape)) == 1 else "
                                     "np.resize(k, shape[-1]).reshape([1] * (len(shape) - 1) + [shape[-1]])",
                                     "spectral_derivatives"),
}

_RUN_MUTANT = """
import importlib.util, sys
import oracle
spec = importlib.util.spec_from_file_location("oracle.mfp", sys.argv[1])
mod = importlib.util.module_from_spec(spec)
sys.modules["oracle.mfp"] = mod
spec.loader.exec_module(mod)
oracle.mfp = mod
import pytest
sys.exit(pytest.main([sys.argv[2], "-q", "-x", "-p", "no:cacheprovider", "-k", sys.argv[3]]))
"""


@pytest.mark.parametrize("name", sorted(MFP_MUTATIONS))
def test_planted_mistake_in_spatial_oracle_fails_a_pin(name, tmp_path):
    orig, bad, sel = MFP_MUTATIONS[name]
    src = open(MFP_SRC).read()
    assert src.count(orig) == 1, "mutation anchor drifted from the spatial oracle source"
    mut = tmp_path / "mfp_mutant.py"
    mut.write_text(src.replace(orig, bad))
    r = subprocess.run([sys.executable, "-c", _RUN_MUTANT, str(mut),
                        os.path.join(ROOT, "tests", "test_oracle_mfp_pins.py"), sel],
                       cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"no pin caught '{name}':\n{r.stdout[-2000:]}{r.stderr[-2000:]}"


# Mistakes planted in the coupled-step oracle (oracle/ns.py; pins in test_oracle_ns_pins.py).
NS_SRC = os.path.join(ROOT, "oracle", "ns.py")
NS_MUTATIONS = {
    "gradient_transposed": ("self.ifft(1j * self.xi[j] * uh[i]) for i in range(d) for j in range(d)",
                            "self.ifft(1j * self.xi[i] * uh[j]) for i in range(d) for j in range(d)",
                            "derivatives"),
    "stress_divergence_sign": ("F = -box.fft(adv) + box.div_tensor(box.fft(tau_grid))",
                               "F = -box.fft(adv) - box.div_tensor(box.fft(tau_grid))", "shear_wave"),
    "first_order_extrapolation": ("2: ((1.5, -2.0, 0.5), (2.0, -1.0))", "2: ((1.5, -2.0, 0.5), (1.0, 0.0))",
                                  "shear_wave"),
    "pressure_dropped": ("ph = np.where(box.xi2 > 0, divXi / safe, 0.0)", "ph = 0.0 * divXi",
                         "exact_solutions or divergence"),
    "viscosity_sign": ("return rhs / (b[0] / dt + nu * box.xi2), ph", "return rhs / (b[0] / dt - nu * box.xi2), ph",
                       "exact_solutions"),
    "band_not_applied": ("    return F * box.band", "    return F", "exact_product"),
    "advection_index": ("adv = np.stack([sum(u[j] * kap[i * d + j] for j in range(d)) for i in range(d)])",
                        "adv = np.stack([sum(u[j] * kap[j * d + i] for j in range(d)) for i in range(d)])",
                        "exact_product or taylor_green"),
}

_RUN_NS_MUTANT = _RUN_MUTANT.replace("oracle.mfp", "oracle.ns")


@pytest.mark.parametrize("name", sorted(NS_MUTATIONS))
def test_planted_mistake_in_coupled_oracle_fails_a_pin(name, tmp_path):
    orig, bad, sel = NS_MUTATIONS[name]
    src = open(NS_SRC).read()
    assert src.count(orig) == 1, "mutation anchor drifted from the coupled-step oracle source"
    mut = tmp_path / "ns_mutant.py"
    mut.write_text(src.replace(orig, bad))
    r = subprocess.run([sys.executable, "-c", _RUN_NS_MUTANT, str(mut),
                        os.path.join(ROOT, "tests", "test_oracle_ns_pins.py"), sel],
                       cwd=ROOT, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"no pin caught '{name}':\n{r.stdout[-2000:]}{r.stderr[-2000:]}"

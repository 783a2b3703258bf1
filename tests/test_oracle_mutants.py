"""The pins must have teeth: plant one plausible mistake at a time in a
temporary copy of the oracle's C source, rebuild it, and check that at least
one pin in test_oracle_pins.py fails for every planted mistake.  The oracle
under oracle/ is never modified; mutants live in a temporary directory."""
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "vp_oracle.c")
HDR = os.path.join(os.path.dirname(oracle.__file__), "vp_oracle.h")

# (name, original text, mutated text)
MUTANTS = [
    ("phase sign ignored", "obs->sign * 2.0 * ORC_PI", "2.0 * ORC_PI"),
    ("w term dropped", "w * pos[j].n1", "0.0 * pos[j].n1"),
    ("gaussian u/v swapped", "double kx = cos(pa) * v + sin(pa) * u;\n  double ky = -sin(pa) * v + cos(pa) * u;\n  return",
     "double kx = cos(pa) * u + sin(pa) * v;\n  double ky = -sin(pa) * u + cos(pa) * v;\n  return"),
    ("hermite index off by one", "sqrt(n / (n + 1.0))", "sqrt((n + 1.0) / (n + 2.0))"),
    ("fourier factor i^n instead of (sign i)^n", "case 1: orc_add(&im, sign * term)", "case 1: orc_add(&im, -sign * term)"),
    ("rotation transposed", "acc += Tj[i][k] * T0[j][k]", "acc += Tj[k][i] * T0[k][j]"),
    ("beam exponent", "exp(-4.0 * log(2.0) * rho * rho", "exp(-log(2.0) * rho * rho"),
    ("spectral index inverted", "pow(nu / nu_ref, alpha)", "pow(nu_ref / nu, alpha)"),
    ("n-1 sign", "lmn[2] = -(l * l + m * m)", "lmn[2] = (l * l + m * m)"),
    ("kappa without the 2", "double kappa = ORC_PI / sqrt(2.0 * log(2.0));", "double kappa = ORC_PI / sqrt(log(2.0));"),
    ("shapelet frame unrotated", "const double up = R[0] * u + R[1] * v + R[2] * w;\n          const double vp = R[3] * u + R[4] * v + R[5] * w;",
     "const double up = u;\n          const double vp = v;"),
    ("hermite normalisation pi^2", "phi[0] = pow(ORC_PI, -0.25)", "phi[0] = pow(ORC_PI, -1.0)"),
    ("envelope imaginary part dropped", "orc_add(&im, Sj * (xr * s + xi * c));", "orc_add(&im, Sj * (xr * s));"),
]

FAST_PINS = [
    pins.test_basis_counts_match_paper,
    pins.test_every_coefficient_reaches_the_envelope,
    pins.test_hermite_matches_scipy_polynomials,
    pins.test_hermite_at_origin_closed_form,
    pins.test_hermite_cramer_bound,
    pins.test_lmn_textbook_formula_and_unit_norm,
    pins.test_rotation_properties,
    pins.test_gauss_envelope_is_dft_of_image_gaussian,
    lambda: pins.test_shapelet_envelope_is_dft_of_image_basis(2, 1),
    lambda: pins.test_shapelet_envelope_is_dft_of_image_basis(1, 0),
    pins.test_shapelet_00_equals_gaussian,
    pins.test_point_at_phase_centre_is_its_flux,
    pins.test_symmetric_point_pair_is_real_cosine,
    pins.test_gaussian_at_phase_centre_and_zero_width_limit,
    pins.test_hermitian_symmetry_linearity_sign_and_channel_scaling,
    pins.test_beam_reduces_to_flat_at_phase_centre_and_attenuates_off_axis,
    pins.test_whole_sum_against_mpmath_brute_force,
]


def _build_mutant(tmp, orig, new):
    src = open(SRC).read()
    assert src.count(orig) == 1, "mutation anchor not unique: %r" % orig
    os.makedirs(tmp, exist_ok=True)
    open(os.path.join(tmp, "vp_oracle.c"), "w").write(src.replace(orig, new))
    shutil.copy(HDR, tmp)
    so = os.path.join(tmp, "liboracle.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-fopenmp", "-shared", "-o", so,
                    os.path.join(tmp, "vp_oracle.c"), "-lm"], check=True, cwd=tmp)
    return so


@pytest.mark.parametrize("name,orig,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(name, orig, new, monkeypatch):
    with tempfile.TemporaryDirectory() as tmp:
        so = _build_mutant(tmp, orig, new)
        monkeypatch.setattr(oracle, "_LIB_PATH", so)
        monkeypatch.setattr(oracle, "_lib", None)
        caught = []
        for pin in FAST_PINS:
            try:
                pin()
            except AssertionError:
                caught.append(getattr(pin, "__name__", "dft"))
                break
        monkeypatch.setattr(oracle, "_lib", None)
    assert caught, "no pin caught the planted mistake: " + name

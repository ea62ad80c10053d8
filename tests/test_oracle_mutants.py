"""Planted mistakes in the oracle must be caught by its pins (CPU only).

Each case builds a copy of oracle.c with one plausible slip -- a dropped or
mis-scaled term of Eq. 2, a sign flip, an off-by-half pixel centring, x and y
swapped, a missing 1/N in Eq. 1, an inverted GSW weight update, a wrong
uniformity formula, a broken adjoint -- swaps it in for the real library and
checks that at least one pin of tests/test_oracle_pins.py now fails.
"""
import ctypes as C
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "lens term dropped": [("t[2] * ORC_PI / (lam * f * f) * (x * x + y * y) + ", "")],
    "lens term doubled": [("t[2] * ORC_PI / (lam * f * f)", "t[2] * 2.0 * ORC_PI / (lam * f * f)")],
    "y grating dropped": [("(x * t[0] + y * t[1])", "(x * t[0])")],
    "x and y swapped": [("(x * t[0] + y * t[1])", "(x * t[1] + y * t[0])")],
    "centring off by half a pixel": [("0.5 * (double)(nx - 1)", "0.5 * (double)nx")],
    "forward sign flipped": [("double a = phi[j] - delta(", "double a = phi[j] + delta(")],
    "backward theta sign": [("lam, f) + theta[m];", "lam, f) - theta[m];")],
    "missing 1/N": [("V[2 * m] = re / (double)N;", "V[2 * m] = re;"),
                    ("V[2 * m + 1] = im / (double)N;", "V[2 * m + 1] = im;")],
    "no wrap to [0, 2 pi)": [("wrap_2pi(atan2(im, re))", "atan2(im, re)")],
    "inverted weight update": [("w[m] *= mean / (tiny ? 1e-12 * mean : a);",
                                "w[m] *= (tiny ? 1e-12 * mean : a) / mean;")],
    "theta update conjugated": [("th[m] = atan2(V[2 * m + 1], V[2 * m]);",
                                 "th[m] = -atan2(V[2 * m + 1], V[2 * m]);")],
    "uniformity formula": [("1.0 - (mx - mn) / (mx + mn)", "(mx - mn) / (mx + mn)")],
    "adjoint real part": [("grad[j] = (im * cos(phi[j]) - re * sin(phi[j]))",
                           "grad[j] = (re * cos(phi[j]) - im * sin(phi[j]))")],
    "loss gradient drops var term": [(" - 2.0 * var / (M * mu * mu * mu)", "")],
    "splitmix constant": [("0xBF58476D1CE4E5B9ULL", "0xBF58476D1CE4E5B8ULL")],
}

# fast pins first; the finite-difference gradient (a few seconds) last
PINS = [
    (pins.test_single_trap_grating_is_dft_ramp, ()),
    (pins.test_single_trap_defocus_is_thin_lens, ()),
    (pins.test_single_trap_full_efficiency, ("gsw", 3)),
    (pins.test_forward_on_fourier_grid_matches_fft2, ()),
    (pins.test_backward_on_fourier_grid_matches_ifft2, ()),
    (pins.test_binary_grating_fourier_coefficient, ()),
    (pins.test_backward_forward_duality, ()),
    (pins.test_stats_definitions, ()),
    (pins.test_splitmix64_published_vector, ()),
    (pins.test_mirror_symmetry_of_symmetric_grid, ()),
    (pins.test_gs_is_monotone_ascent, ()),
    (pins.test_gsw_weighted_ascent_inequality, ()),
    (pins.test_gsw_converges_to_uniform, ()),
    (pins.test_brute_force_8x8, ("gsw",)),
    (pins.test_brute_force_4x4_mpmath, ()),
    (pins.test_adjoint_of_linear_functional, ()),
    (pins.test_loss_gradient_matches_central_differences, ()),
]


def test_unmutated_source_passes_all_pins():
    for fn, args in PINS:
        fn(*args)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path, monkeypatch):
    src = open(SRC).read()
    for old, new in MUTANTS[name]:
        assert src.count(old) == 1, f"mutation anchor not unique/found: {old!r}"
        src = src.replace(old, new)
    cfile, sofile = tmp_path / "mut.c", tmp_path / "libmut.so"
    cfile.write_text(src)
    subprocess.check_call(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                           "-o", str(sofile), str(cfile), "-lm"])
    monkeypatch.setattr(oracle, "_lib", oracle.configure(C.CDLL(str(sofile))))
    caught = None
    for fn, args in PINS:
        try:
            fn(*args)
        except Exception as e:  # an assertion or a downstream numerical failure
            caught = f"{fn.__name__}: {type(e).__name__}"
            break
    assert caught is not None, f"planted mistake '{name}' passed every pin"

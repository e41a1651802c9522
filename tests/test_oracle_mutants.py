"""The pins are strong enough: each plausible mistake, planted in a copy of the
oracle's C source and compiled on the CPU, makes at least one pin fail."""
import os

import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "tso_oracle.c")

# name -> list of (original text, planted mistake)
MUTANTS = {
    "printed -i sign of the rotation": [("(-s * bi", "(s * bi"), ("(s * br", "(-s * br"),
                                         ("(-s * ai", "(s * ai"), ("(s * ar", "(-s * ar")],
    "dropped 1 - cos term": [("*d = 2.0 * half * half;", "*d = 0.0;")],
    "sin^2 without the factor 2": [("*d = 2.0 * half * half;", "*d = half * half;")],
    "half factors act for dt": [("double h = 0.5 * dt;", "double h = dt;")],
    "diagonal constant dropped": [("    double eps0 = hbar * hbar / (mass * dx * dx) + hbar * hbar / (mass * dy * dy);\n    double sx",
                                   "    double eps0 = 0.0;\n    double sx")],
    "phase sign": [("psi[2 * l] = re * c + im * s;", "psi[2 * l] = re * c - im * s;"),
                   ("psi[2 * l + 1] = im * c - re * s;", "psi[2 * l + 1] = im * c + re * s;")],
    "potential ignored": [("double phi = dt * (V[l] + eps0) / hbar;", "double phi = dt * eps0 / hbar;")],
    "even and odd factors swapped": [("sweep_x(nx, ny, bc, 1, sx, dxc, psi);  /* Ox(h) */\n    sweep_y(nx, ny, bc, 1, sy, dyc, psi);  /* Oy(h) */\n    sweep_x(nx, ny, bc, 0",
                                      "sweep_x(nx, ny, bc, 0, sx, dxc, psi);  /* Ox(h) */\n    sweep_y(nx, ny, bc, 0, sy, dyc, psi);  /* Oy(h) */\n    sweep_x(nx, ny, bc, 1")],
    "wrap pair missing along x": [("            if (k == nx) {\n                if (bc == TSO_BC_CLOSED) continue;\n                k = 0;",
                                   "            if (k == nx) {\n                continue;\n                k = 0;")],
    "y factors use the x spacing": [("block_coeffs(h, Jy, hbar, &sy, &dyc);", "block_coeffs(h, Jx, hbar, &sy, &dyc);")],
    "energy hop sign": [("hr -= Jx * psi[2 * m];", "hr += Jx * psi[2 * m];")],
    "norm drops the imaginary part": [("sn += pr * pr + pi * pi;", "sn += pr * pr;")],
    "time-dependent modulation ignored": [("Vn[l] = V0[l] + f[n] * W[l];", "Vn[l] = V0[l] + 0.0 * W[l];")],
    "modulation lags one step": [("Vn[l] = V0[l] + f[n] * W[l];", "Vn[l] = V0[l] + f[n > 0 ? n - 1 : 0] * W[l];")],
    "modulation without the time step": [("Vn[l] = V0[l] + f[n] * W[l];", "Vn[l] = V0[l] + f[n] * W[l] / dt;")],
    "3D: the z spacing takes the y one": [("hbar * hbar / (2.0 * mass * dz * dz)};\n    double eps0 = 2.0 * (J[0] + J[1] + J[2]);\n    double sa[3]",
                                           "hbar * hbar / (2.0 * mass * dy * dy)};\n    double eps0 = 2.0 * (J[0] + J[1] + J[2]);\n    double sa[3]")],
    "3D: diagonal misses the z constant": [("double eps0 = 2.0 * (J[0] + J[1] + J[2]);\n    double sa[3]",
                                            "double eps0 = 2.0 * (J[0] + J[1]);\n    double sa[3]")],
    "3D: opening odd z factor missing": [("for (int a = 0; a < 3; ++a) sweep3(nx, ny, nz, bc, a, 1, sa[a], da[a], psi);  /* O(h) */",
                                          "for (int a = 0; a < 2; ++a) sweep3(nx, ny, nz, bc, a, 1, sa[a], da[a], psi);  /* O(h) */")],
    "energy misses y neighbours": [("hr -= Jy * psi[2 * m];", "hr -= 0.0 * psi[2 * m];"),
                                   ("hi -= Jy * psi[2 * m + 1];", "hi -= 0.0 * psi[2 * m + 1];")],
}

CHECKS = [
    lambda: pins.test_single_factor_equals_dense_expm((6, 4), "periodic", "x", 1),
    lambda: pins.test_single_factor_equals_dense_expm((6, 4), "periodic", "y", 0),
    lambda: pins.test_single_factor_equals_dense_expm((6, 4), "periodic", "P", 0),
    lambda: pins.test_step_equals_dense_factor_product((6, 4), "periodic"),
    lambda: pins.test_step_equals_dense_factor_product((5, 3), "closed"),
    lambda: pins.test_error_shrinks_as_dt_squared((6, 4), "periodic"),
    lambda: pins.test_bloch_closed_form((16, 16), 7),
    lambda: pins.test_plane_wave_energy((3, 1)),
    lambda: pins.test_energy_equals_dense_expectation((6, 4), "periodic"),
    lambda: pins.test_td_error_shrinks_as_dt_squared((6, 4), "periodic"),
    lambda: pins.test_td_step_equals_dense_product_of_frozen_steps(),
    lambda: pins.test_3d_step_equals_dense_factor_product((4, 4, 4), "periodic"),
    lambda: pins.test_3d_separable_problem_is_tensor_product_of_1d_runs(),
]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path, monkeypatch):
    text = open(SRC).read()
    for old, new in MUTANTS[name]:
        assert old in text, (name, old)
        text = text.replace(old, new)
    src = tmp_path / "mutant.c"
    src.write_text(text)
    lib = oracle.load_library(oracle.compile_library(str(src), str(tmp_path / "libmutant.so")))
    monkeypatch.setattr(oracle, "_lib", lib)
    caught = 0
    for check in CHECKS:
        try:
            check()
        except (AssertionError, ValueError):
            caught += 1
    assert caught > 0, f"no pin catches: {name}"


def test_unmutated_copy_passes_every_check(tmp_path, monkeypatch):
    src = tmp_path / "same.c"
    src.write_text(open(SRC).read())
    lib = oracle.load_library(oracle.compile_library(str(src), str(tmp_path / "libsame.so")))
    monkeypatch.setattr(oracle, "_lib", lib)
    for check in CHECKS:
        check()

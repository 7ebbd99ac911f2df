"""Planted mistakes in a copy of the noise-normalisation oracle must each
fail a pin (CPU only). Applied to a temporary copy of oracle/nn_oracle.cpp,
compiled and loaded by tests/test_nn_oracle_pins.py in a subprocess."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nn_oracle.cpp")

MUTANTS = {
    "centre_upper_middle": ("k.centre = k.lo + (k.hi - k.lo) / 2;",
                            "k.centre = k.lo + (k.hi - k.lo + 1) / 2;"),
    "window_short_on_the_left": ("*a = std::max<int64_t>(0, centre - r);",
                                 "*a = std::max<int64_t>(0, centre - r + 1);"),
    "window_clipped_one_short": ("*b = std::min<int64_t>(n - 1, centre + r);",
                                 "*b = std::min<int64_t>(n - 2, centre + r);"),
    "y_window_takes_z_radius": ("window_of(ky.centre, rxy, ny, &y0, &y1);",
                                "window_of(ky.centre, rz, ny, &y0, &y1);"),
    "block_end_overruns": ("k.hi = std::min(n, (b + 1) * g) - 1;",
                           "k.hi = std::min(n, (b + 1) * g);"),
    "negative_includes_zero": ("if (range == kRangeNeg) return v < 0.0;",
                               "if (range == kRangeNeg) return v <= 0.0;"),
    "median_upper_only": ("return kMadToSigma * (hi == lo ? v_lo : 0.5 * (v_lo + v_hi));",
                          "return kMadToSigma * v_hi;"),
    "multiply_not_divide": ("(float)(d / s)", "(float)(d * s)"),
    "unusable_block_not_blanked": ("Y[i] = (usable && std::isfinite(d))",
                                   "Y[i] = (std::isfinite(d))"),
    "std_n_minus_1": ("return std::sqrt(sum / (double)m);",
                      "return std::sqrt(sum / (double)(m > 1 ? m - 1 : 1));"),
    "mad_constant": ("kMadToSigma = 1.4826;", "kMadToSigma = 1.4826022;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/found"
    mut = tmp_path / "mutant.cpp"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                    "-ffp-contract=off", str(mut), "-o", str(lib)], check=True)
    env = dict(os.environ, NN_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_nn_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"

"""Planted mistakes in a copy of the oracle must each fail a pin (CPU only).

Every mutant is a plausible slip (a dropped term, a wrong sign, an index off
by one, a transposed operand, a wrong constant). It is applied to a temporary
copy of oracle/sc_oracle.cpp, compiled, and the pin suite is run against the
copy in a subprocess; the suite must fail. The committed oracle is untouched.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sc_oracle.cpp")

MUTANTS = {
    "gauss_radius_floor": ("(int64_t)std::floor(4.0 * sigma_g + 0.5);",
                           "(int64_t)std::floor(4.0 * sigma_g);"),
    "gauss_unnormalised": ("for (double &v : h) v /= sum;", "for (double &v : h) v /= 1.0;"),
    "gauss_variance_factor": ("std::exp(-(double)(k * k) / (2.0 * sigma_g * sigma_g));",
                              "std::exp(-(double)(k * k) / (sigma_g * sigma_g));"),
    "gauss_y_pass_dropped": ("        taps_axis(S, nx, ny, nz, 1, taps);\n", ""),
    "gauss_edge_replicated": ("if (k >= 0 && k < len) acc += h[(size_t)(j + R)] * in[k];",
                              "acc += h[(size_t)(j + R)] * in[k < 0 ? 0 : (k >= len ? len - 1 : k)];"),
    "divisor_2r": ("const double width = (double)(2 * r + 1);",
                   "const double width = (double)(2 * r);"),
    "window_off_by_one": ("for (int64_t j = -r; j <= r; ++j) {",
                          "for (int64_t j = -r; j < r; ++j) {"),
    "periodic_edges": ("if (k >= 0 && k < len) acc += in[k];",
                       "acc += in[(k + len) % len];"),
    "reflected_operand": ("if (k >= 0 && k < len) acc += in[k];",
                          "if (k >= 0 && k < len) acc += in[len - 1 - k];"),
    "y_axis_dropped": ("        smooth_axis(S, nx, ny, nz, 1, n_it, r);\n", ""),
    "spectral_radius": ("smooth_axis(S, nx, ny, nz, 2, 1, (width - 1) / 2);",
                        "smooth_axis(S, nx, ny, nz, 2, 1, (width + 1) / 2);"),
    "replacement_sign_lost": ("y = std::copysign(rv, d);", "y = rv;"),
    "replacement_ignores_sigma0": ("const double rv = repl * sigma0;",
                                   "const double rv = repl;"),
    "mad_constant": ("kMadToSigma = 1.4826;", "kMadToSigma = 1.4826022;"),
    "median_upper_only": ("hi == lo ? v_lo : 0.5 * (v_lo + v_hi);",
                          "hi == lo ? v_lo : v_hi;"),
    "negative_includes_zero": ("if (range == kRangeNeg) return s < 0.0;",
                               "if (range == kRangeNeg) return s <= 0.0;"),
    "std_n_minus_1": ("*sigma = std::sqrt(sum / (double)m);",
                      "*sigma = std::sqrt(sum / (double)(m > 1 ? m - 1 : 1));"),
    "clip_not_strict": ("if (std::fabs(s) > T) mask[i] = 1;",
                        "if (std::fabs(s) >= T) mask[i] = 1;"),
    "blanked_not_restored": ("if (!std::isfinite(X[i])) S[i] = NAN;",
                             "if (!std::isfinite(X[i])) S[i] = S[i];"),
    "plan_tie_to_smaller_n": ("(d == best_d && (n > best_n ||",
                              "(d == best_d && (n < best_n ||"),
    "fwhm_factor": ("fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));\n    const double target",
                    "fwhm / std::sqrt(2.0 * std::log(2.0));\n    const double target"),
    "gauss_fwhm_factor": ("fwhm / (2.0 * std::sqrt(2.0 * std::log(2.0)));\n    const int64_t R",
                          "fwhm / std::sqrt(2.0 * std::log(2.0));\n    const int64_t R"),
    "union_dropped": ("if (mask_prev) std::memcpy(mask_out, mask_prev, (size_t)N);\n"
                      "    else std::memset(mask_out, 0, (size_t)N);\n    return noise_and_clip(",
                      "if (false) std::memcpy(mask_out, mask_prev, (size_t)N);\n"
                      "    else std::memset(mask_out, 0, (size_t)N);\n    return noise_and_clip("),
    # the boundary band excuses mask differences in every parity test
    "band_too_wide": ("kBandWidth = 1e-5;", "kBandWidth = 1e-2;"),
    "band_too_narrow": ("kBandWidth = 1e-5;", "kBandWidth = 1e-6;"),
    "band_absolute_units": ("std::fabs(std::fabs(s) / (*sigma_k) - t) <= kBandWidth",
                            "std::fabs(std::fabs(s) - T) <= kBandWidth"),
    # the subsampled / given-noise step
    "sub_stride_offset": ("if ((i / ncol) % plane_stride != 0) Ssub[(size_t)i] = NAN;",
                          "if ((i / ncol) % plane_stride != 1) Ssub[(size_t)i] = NAN;"),
    "sub_clip_not_strict": ("if (std::fabs(s) > T) mask_out[i] = 1;",
                            "if (std::fabs(s) >= T) mask_out[i] = 1;"),
    "sub_band_absolute": ("std::fabs(std::fabs(s) / sig - t) <= kBandWidth",
                          "std::fabs(std::fabs(s) - T) <= kBandWidth"),
    "sub_union_dropped": ("    if (mask_prev) std::memcpy(mask_out, mask_prev, (size_t)N);\n    else std::memset(mask_out, 0, (size_t)N);\n    double sig",
                          "    std::memset(mask_out, 0, (size_t)N);\n    double sig"),
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
    env = dict(os.environ, SC_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"

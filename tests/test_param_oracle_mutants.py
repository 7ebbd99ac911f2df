"""Planted mistakes in a copy of the parameterisation / reliability oracle
(oracle/param.py) must each fail a pin (CPU only)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "param.py")

MUTANTS = {
    "omega_without_4ln2": ("return math.pi * a * b / (4.0 * math.log(2.0))",
                           "return math.pi * a * b / 4.0"),
    "flux_err_without_sqrt_n": ("flux_err = np.sqrt(count) * channel_width",
                                "flux_err = count * channel_width"),
    "flux_err_full_omega": ("sigma_rms / math.sqrt(omega)", "sigma_rms / omega"),
    "flux_times_omega": ("flux = channel_width / omega * s", "flux = channel_width * omega * s"),
    "nan_voxels_counted": ("ok = (lab > 0) & (lab <= n) & np.isfinite(x)",
                           "ok = (lab > 0) & (lab <= n)"),
    "covariance_ddof_0": ("cov = np.cov(vn.T, ddof=1) * scale * scale",
                          "cov = np.cov(vn.T, ddof=0) * scale * scale"),
    "scale_not_squared": ("cov = np.cov(vn.T, ddof=1) * scale * scale",
                          "cov = np.cov(vn.T, ddof=1) * scale"),
    "negative_vector_uses_peak": ("return np.log10(np.stack([-p[\"min\"], -p[\"sum\"], -p[\"mean\"]], axis=1))",
                                  "return np.log10(np.stack([-p[\"peak\"], -p[\"sum\"], -p[\"mean\"]], axis=1))"),
    "reliability_not_clipped": ("R[ev] = np.maximum(0.0, (P - N) / P)", "R[ev] = (P - N) / P"),
    "snr_threshold_strict": ("(p[\"snr\"] >= snr_threshold)", "(p[\"snr\"] > snr_threshold)"),
    "centroid_unweighted": ("sx = np.bincount(lab, weights=v * px, minlength=n + 1)[1:]",
                            "sx = np.bincount(lab, weights=px * 1.0, minlength=n + 1)[1:]"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/found"
    mut = tmp_path / "param_mutant.py"
    mut.write_text(src.replace(old, new))
    env = dict(os.environ, PARAM_ORACLE_FILE=str(mut))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_param_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"

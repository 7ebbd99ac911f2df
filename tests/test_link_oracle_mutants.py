"""Planted mistakes in a copy of the linker oracle must each fail a pin (CPU
only). Applied to a temporary copy of oracle/link_oracle.cpp, compiled and
loaded by tests/test_link_oracle_pins.py in a subprocess."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "link_oracle.cpp")

MUTANTS = {
    "box_not_ellipsoid": ("if (rxy > 0 && rz > 0) in = sxy * c + sz * a <= a * c;",
                          "if (rxy > 0 && rz > 0) in = true;"),
    "strict_radius": ("if (rxy > 0 && rz > 0) in = sxy * c + sz * a <= a * c;",
                      "if (rxy > 0 && rz > 0) in = sxy * c + sz * a < a * c;"),
    "radius_axes_swapped": ("if (rxy > 0 && rz > 0) in = sxy * c + sz * a <= a * c;",
                            "if (rxy > 0 && rz > 0) in = sxy * a + sz * c <= a * c;"),
    "planar_radius_strict": ("else if (rxy > 0) in = sz == 0 && sxy <= a;",
                             "else if (rxy > 0) in = sz == 0 && sxy < a;"),
    "x_offsets_one_short": ("for (int dx = -rxy; dx <= rxy; ++dx) {",
                            "for (int dx = -rxy; dx < rxy; ++dx) {"),
    "extent_without_plus_one": ("const int64_t ex = b.x1 - b.x0 + 1, ey = b.y1 - b.y0 + 1,",
                                "const int64_t ex = b.x1 - b.x0, ey = b.y1 - b.y0 + 1,"),
    "min_filter_strict": ("bool keep = ex >= min_xy && ey >= min_xy && ez >= min_z;",
                          "bool keep = ex > min_xy && ey >= min_xy && ez >= min_z;"),
    "y_extent_ignored": ("bool keep = ex >= min_xy && ey >= min_xy && ez >= min_z;",
                         "bool keep = ex >= min_xy && ez >= min_z;"),
    "max_z_ignored": ("if (max_z > 0 && ez > max_z) keep = false;", ""),
    "dropped_keep_their_label": ("if (!keep) continue;", "if (!keep && false) continue;"),
    "count_not_incremented": ("            b.count += 1;\n", ""),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique/found"
    mut = tmp_path / "mutant.cpp"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", str(mut), "-o", str(lib)],
                   check=True)
    env = dict(os.environ, LINK_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_link_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"

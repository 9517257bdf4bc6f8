"""Strength of the oracle's pins: plausible mistakes planted in a copy of the
oracle must each fail at least one pin.

Each case copies the oracle package into a temporary directory, applies one
textual change to its C source, builds it there and runs the oracle's pin
modules against that copy in a fresh interpreter (the copy comes first on the
import path). The unmodified copy must pass the same pins (control), so a
failing mutant fails because of its change. Nothing here touches the GPU
library.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = [os.path.join(ROOT, "tests", f) for f in (
    "test_oracle_pins.py", "test_oracle_geometry.py", "test_oracle_cylinder.py",
    "test_oracle_sart.py")]

# name -> (text in gjp_oracle.c, replacement)
MUTANTS = {
    # Eq. 13: the weight of the lower neighbour swapped with the upper one's
    "linear_weight_swapped": ("return 1.0 - d;", "return d;"),
    # Eq. 14: a wrong cubic coefficient
    "spline_coefficient": ("1.0 - 3.0 * d * d + 2.0 * d * d * d",
                           "1.0 - 3.0 * d * d + 3.0 * d * d * d"),
    # Eq. 9: the upper neighbour weighted by w(1 - |t|) instead of w(|t|)
    "complementary_weight": ("const double a = fabs(t);",
                             "const double a = t < 0.0 ? 1.0 + t : t;"),
    # Eq. 3: ties to the highest axis index
    "argmax_tie_rule": ("if (fabs(r[k]) > fabs(r[m])) m = k;",
                        "if (fabs(r[k]) >= fabs(r[m])) m = k;"),
    # in-volume test read as the grid's own extent instead of the padded domain
    "strict_boundary": ("if (!(q[k] > -1.0 && q[k] < (double)g->n[k])) return 0;",
                        "if (!(q[k] >= 0.0 && q[k] <= (double)(g->n[k] - 1))) return 0;"),
    # Algorithm 1's loop bounds: the first plane dropped from the forward
    "sample_range": ("  for (int i = 0; i < g->n[ray.m]; ++i) {\n    double q[3];\n"
                     "    if (!plane_point(g, &ray, i, q)) continue;\n    sum +=",
                     "  for (int i = 1; i < g->n[ray.m]; ++i) {\n    double q[3];\n"
                     "    if (!plane_point(g, &ray, i, q)) continue;\n    sum +="),
    # grid convention: voxel k centred at k + 1/2 instead of k
    "grid_offset": ("out[k] = (w[k] - g->ctr[k]) / g->vs[k] + (double)(g->n[k] - 1) * 0.5;",
                    "out[k] = (w[k] - g->ctr[k]) / g->vs[k] + (double)g->n[k] * 0.5;"),
    # the step length squared instead of its square root
    "step_length": ("ray->len = sqrt(q);", "ray->len = q;"),
    # Eq. 5 with the wrong sign of the offset
    "offset_sign": ("(-ray->s[m] + (double)i) * ray->rt[k]", "(ray->s[m] + (double)i) * ray->rt[k]"),
    # Eq. 7: one of the four in-plane neighbours dropped
    "dropped_neighbour": ("for (long long ja = base_a; ja <= base_a + 1; ++ja) {\n"
                          "    const double ha = kernel_1d(g->weight, q[a] - (double)ja);\n"
                          "    for (long long jb = base_b; jb <= base_b + 1; ++jb) {\n"
                          "      const double hb = kernel_1d(g->weight, q[b] - (double)jb);\n"
                          "      long long j[3];\n      j[m]",
                          "for (long long ja = base_a; ja <= base_a + 1; ++ja) {\n"
                          "    const double ha = kernel_1d(g->weight, q[a] - (double)ja);\n"
                          "    for (long long jb = base_b; jb <= base_b; ++jb) {\n"
                          "      const double hb = kernel_1d(g->weight, q[b] - (double)jb);\n"
                          "      long long j[3];\n      j[m]"),
    # the adjoint missing one axis's weight
    "adjoint_weight": ("vol[idx] += scaled * (ha * hb);", "vol[idx] += scaled * ha;"),
    # detector axes swapped in the pixel position
    "detector_axes": ("d[k] = det00[k] + (double)iu * du[k] + (double)iv * dv[k];",
                      "d[k] = det00[k] + (double)iv * du[k] + (double)iu * dv[k];"),
}


def _run_pins(copy_root):
    env = dict(os.environ)
    env["PYTHONPATH"] = os.pathsep.join([copy_root, ROOT])
    env["OMP_NUM_THREADS"] = env.get("OMP_NUM_THREADS", "4")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
           "-m", "not gpu", *PINS]
    # cwd is the copy: `python -m` puts the working directory first on the path
    return subprocess.run(cmd, cwd=copy_root, env=env, capture_output=True, text=True,
                          timeout=600)


def _make_copy(tmp_path, mutation=None):
    root = str(tmp_path)
    dst = os.path.join(root, "oracle")
    shutil.copytree(os.path.join(ROOT, "oracle"), dst,
                    ignore=shutil.ignore_patterns("*.so", "*.so.tmp", "__pycache__"))
    if mutation is not None:
        old, new = mutation
        src = os.path.join(dst, "gjp_oracle.c")
        text = open(src).read()
        assert text.count(old) == 1, f"mutation site not unique or missing: {old!r}"
        open(src, "w").write(text.replace(old, new))
    subprocess.check_call([sys.executable, os.path.join(dst, "build.py")], cwd=root,
                          stdout=subprocess.DEVNULL)
    return root


def test_unmodified_copy_passes_pins(tmp_path):
    r = _run_pins(_make_copy(tmp_path))
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-2000:]
    # the copy, not the repository's oracle, was the one imported
    assert "passed" in r.stdout


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_fails_a_pin(tmp_path, name):
    r = _run_pins(_make_copy(tmp_path, MUTANTS[name]))
    assert r.returncode == 1, f"mutant {name} passed every pin:\n" + r.stdout[-3000:]
    assert "failed" in r.stdout

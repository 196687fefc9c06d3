"""Host build of the position wrap and cell index used by the key kernels.

The forward reads its input check only after the cell keys of a speculative
attempt are computed, so the keys must stay in range for any input: a
non-finite or huge coordinate maps to the origin (cell 0), and every finite
coordinate to [0, L) and a cell in [0, G). The two helpers are
__host__ __device__; this compiles them for the host alone and checks them
on edge values and on random coordinates against floor-mod arithmetic.
"""
import math
import os
import subprocess

import numpy as np

from tests.conftest import ROOT

SRC = r"""
#include <cstdio>
#include <cstdlib>
#include "crk_device.h"
int main(int argc, char** argv) {
  const double L = atof(argv[1]);
  const int G = atoi(argv[2]);
  double x;
  while (scanf("%lf", &x) == 1) {
    const double t = crk::wrap_pos(x, L);
    printf("%.17g %d\n", t, crk::cell_coord(t, (double)G / L, G));
  }
  return 0;
}
"""


def _run(tmp_path, L, G, xs):
    exe = tmp_path / "wrap"
    if not exe.exists():
        src = tmp_path / "wrap.cpp"
        src.write_text(SRC)
        subprocess.check_call(["/opt/rocm/bin/hipcc", "-x", "hip", "--cuda-host-only", "-O2",
                               "-I", os.path.join(ROOT, "paper_2511_21921_amd", "csrc"),
                               str(src), "-o", str(exe)], stderr=subprocess.DEVNULL)
    inp = "\n".join(repr(float(v)) if math.isfinite(v) else
                    ("nan" if math.isnan(v) else ("inf" if v > 0 else "-inf")) for v in xs)
    out = subprocess.run([str(exe), repr(L), str(G)], input=inp, capture_output=True, text=True,
                         check=True).stdout.split()
    return np.array(out[0::2], dtype=np.float64), np.array(out[1::2], dtype=np.int64)


def test_nonfinite_and_huge_coordinates_map_to_cell_zero(tmp_path):
    xs = [math.nan, -math.nan, math.inf, -math.inf, 1e300, -1e300, 1.7e308, -1.7e308]
    for L, G in ((1.0, 1024), (3.5, 17), (1e-3, 2)):
        t, c = _run(tmp_path, L, G, xs)
        assert np.all(t == 0.0) and np.all(c == 0), (L, G, t, c)


def test_finite_coordinates_wrap_into_the_box(tmp_path):
    rng = np.random.default_rng(5)
    for L, G in ((1.0, 1024), (3.5, 17), (1e-3, 2), (1.0, 1)):
        xs = np.concatenate([rng.uniform(-10 * L, 10 * L, 2000),
                             [0.0, -0.0, L, -L, 2 * L, np.nextafter(L, 0), -1e-300, 1e-300,
                              np.nextafter(0.0, -1.0) * 1e16]])
        t, c = _run(tmp_path, L, G, xs)
        assert np.all((t >= 0) & (t < L)), (L, G)
        assert np.all((c >= 0) & (c < G)), (L, G)
        ref = np.mod(xs, L)
        ok = np.isclose(t, ref, rtol=0, atol=4e-16 * 10 * L) | np.isclose(t + L, ref, atol=1e-15 * L)
        assert np.all(ok | (ref >= L * (1 - 1e-15))), (L, G)
        assert np.all(c == np.minimum((t * (G / L)).astype(np.int64), G - 1))

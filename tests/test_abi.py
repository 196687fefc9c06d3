"""Host-only checks of the C ABI: the library loads, exports every function
that include/crk.h declares, and the ctypes mirrors match the C layouts."""
import ctypes as C
import os
import re
import subprocess

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "crk.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(crk_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def crk():
    from paper_2511_21921_amd import crk
    if not os.path.exists(crk.LIB_PATH):
        from paper_2511_21921_amd import build
        build.build()
    return crk


def test_library_exports_every_declared_symbol(crk):
    L = crk.lib()
    names = _declared()
    assert set(names) == set(crk.EXPORTS)
    for name in names:
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", crk.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for name in names:
        assert re.search(r"\bT %s\b" % name, out), name


def test_struct_layouts_match_header(crk, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "crk.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(crk_params), offsetof(crk_params, h_rtol),
         offsetof(crk_params, check_finite), offsetof(crk_params, search), sizeof(crk_stats),
         offsetof(crk_stats, grid), offsetof(crk_stats, speculative),
         offsetof(crk_stats, n_candidates), offsetof(crk_stats, n_searched));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(t) for t in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(crk.crk_params), crk.crk_params.h_rtol.offset,
            crk.crk_params.check_finite.offset, crk.crk_params.search.offset,
            C.sizeof(crk.crk_stats), crk.crk_stats.grid.offset, crk.crk_stats.speculative.offset,
            crk.crk_stats.n_candidates.offset, crk.crk_stats.n_searched.offset]
    assert got == want


def test_default_params_host_only(crk):
    p = crk.crk_params()
    crk.lib().crk_default_params(C.byref(p), crk.FP64)
    assert p.box == 1.0 and p.precision == crk.FP64 and p.h_rtol == 1e-13
    assert abs(p.gamma - 5 / 3) < 1e-15 and p.alpha == 1.0 and p.beta == 2.0


@pytest.mark.parametrize("field,value", [("box", 0.0), ("box", -1.0), ("n_h", 0.5),
                                         ("kernel", 7), ("precision", 3), ("h_mode", 2),
                                         ("h_rtol", 0.0), ("gamma", 1.0)])
def test_create_rejects_bad_params_without_device(crk, field, value):
    p = crk.crk_params()
    crk.lib().crk_default_params(C.byref(p), crk.FP32)
    setattr(p, field, value)
    h = C.c_void_p()
    assert crk.lib().crk_create(C.byref(h), C.byref(p)) == -1
    assert not h.value


def test_null_context_is_rejected(crk):
    L = crk.lib()
    assert L.crk_destroy(None) == 0
    assert L.crk_reserve(None, 10) == -1
    assert L.crk_forward(None, None, 0, *([None] * 14), None) == -1
    assert L.crk_backward(None, None, 0, *([None] * 6)) == -1
    assert L.crk_kdk_step(None, None, 0, 1e-3, 0.5, *([None] * 14), None) == -1
    assert L.crk_hkdk_step(None, None, 0, 1e-3, 0.5, *([None] * 17), None) == -1
    assert L.crk_cooling_table(None, None, 2, 0.0, 0.1, None) == -1
    assert L.crk_cool(None, None, 0, 1.0, None, None) == -1
    assert L.crk_deposit(None, None, 0, *([None] * 7), 0, *([None] * 5), 2.0, 1.0, 1.0,
                         None, None, None) == -1

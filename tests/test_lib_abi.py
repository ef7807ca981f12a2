"""Host-only checks of the C ABI: the library builds, loads and exports every
entry point the header declares, and the binding's grid struct matches the
header's layout.  No GPU call is made."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppmb.h")


def _lib_path():
    from paper_1810_13416_amd import ppmb
    if not os.path.exists(ppmb.LIB_PATH):
        from paper_1810_13416_amd import build
        build.build()
    return ppmb.LIB_PATH


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ppmb_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    from paper_1810_13416_amd import ppmb
    assert set(declared_functions()) == set(ppmb.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(_lib_path())
    missing = [f for f in declared_functions() if not hasattr(L, f)]
    assert not missing, missing


def test_library_has_no_torch_dependency():
    # the NEEDED entries of the dynamic section, independent of how the
    # loader would resolve them in this environment
    out = subprocess.run(["readelf", "-d", _lib_path()], capture_output=True, text=True).stdout
    needed = [l for l in out.splitlines() if "(NEEDED)" in l]
    assert needed and any("amdhip64" in l for l in needed)
    assert not any("torch" in l or "c10" in l for l in needed), needed


def test_status_strings_without_gpu():
    L = ctypes.CDLL(_lib_path())
    L.ppmb_status_string.restype = ctypes.c_char_p
    L.ppmb_status_string.argtypes = [ctypes.c_int]
    assert L.ppmb_status_string(0) == b"ok"
    assert L.ppmb_status_string(-4) == b"non-physical state"
    assert L.ppmb_status_string(-5) == b"time step above the Courant limit"


def test_setters_reject_a_null_context_without_gpu():
    # argument errors are reported at once, before any HIP call
    L = ctypes.CDLL(_lib_path())
    D = ctypes.POINTER(ctypes.c_double)
    L.ppmb_set_gravity.argtypes = [ctypes.c_void_p, ctypes.c_int, D, ctypes.c_int]
    L.ppmb_set_heating.argtypes = [ctypes.c_void_p, ctypes.c_int, D, ctypes.c_int]
    L.ppmb_set_cfl_check.argtypes = [ctypes.c_void_p, ctypes.c_double]
    g = (ctypes.c_double * 4)(0.0, 0.0, -1.0, 0.0)
    assert L.ppmb_set_gravity(None, 1, g, 3) == -1
    assert L.ppmb_set_heating(None, 1, g, 3) == -1
    assert L.ppmb_set_cfl_check(None, 1.0) == -1


def test_grid_struct_layout_matches_header():
    from paper_1810_13416_amd.ppmb import Grid
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "ppmb.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(ppmb_grid), offsetof(ppmb_grid, dx),
         offsetof(ppmb_grid, gamma), offsetof(ppmb_grid, sphere_r), offsetof(ppmb_grid, grav),
         offsetof(ppmb_grid, heat), offsetof(ppmb_grid, smooth_detect));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        vals = [int(v) for v in subprocess.check_output([exe]).split()]
    got = [ctypes.sizeof(Grid), Grid.dx.offset, Grid.gamma.offset, Grid.sphere_r.offset,
           Grid.grav.offset, Grid.heat.offset, Grid.smooth_detect.offset]
    assert vals == got


def test_grid2d_struct_layout_matches_header():
    from paper_1810_13416_amd.ppmb import Grid2D
    src = r"""
#include <stdio.h>
#include <stddef.h>
#include "ppmb.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(ppmb_ppb2d_grid), offsetof(ppmb_ppb2d_grid, dx),
         offsetof(ppmb_ppb2d_grid, origin), offsetof(ppmb_ppb2d_grid, centre),
         offsetof(ppmb_ppb2d_grid, omega));
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        vals = [int(v) for v in subprocess.check_output([exe]).split()]
    got = [ctypes.sizeof(Grid2D), Grid2D.dx.offset, Grid2D.origin.offset, Grid2D.centre.offset,
           Grid2D.omega.offset]
    assert vals == got


def test_binding_refuses_to_run_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_1810_13416_amd import ppmb, problems
    with pytest.raises(ppmb.PPMBError):
        ppmb.Sim(problems.uniform().params)
    with pytest.raises(ppmb.PPMBError):
        ppmb.PPB2D((8, 8), 0.1, (0, 0), (0.4, 0.4), 1.0)


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1810_13416_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "ppmb_oracle" not in text, f

"""The C ABI: the library loads on any host and exports every function that
include/covox.h declares (no device calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "covox.h")
LIB = os.path.join(ROOT, "paper_2410_21149_amd", "libcovox.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(covox_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2410_21149_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_function_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings_and_defaults(lib):
    lib.covox_status_string.restype = ctypes.c_char_p
    for code, name in [(0, b"COVOX_OK"), (-1, b"COVOX_EINVAL"), (-2, b"COVOX_EPOOL_FULL"),
                       (-3, b"COVOX_ETABLE_FULL"), (-4, b"COVOX_EHIP"), (-5, b"COVOX_EDEGENERATE"),
                       (1, b"COVOX_NOT_CONVERGED"), (42, b"COVOX_UNKNOWN")]:
        assert lib.covox_status_string(code) == name
    import importlib.util
    spec = importlib.util.spec_from_file_location("_b", os.path.join(ROOT, "paper_2410_21149_amd", "covox.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    p = mod.default_params()
    assert p.voxel_size == 0.05 and p.trunc_vox == 4 and p.d_max == 2.0 and p.max_iter == 30
    assert p.tol_rho == 1e-7 and p.tol_theta == 1e-8 and p.n_min == 100


def test_create_rejects_bad_params(lib):
    import importlib.util
    spec = importlib.util.spec_from_file_location("_b2", os.path.join(ROOT, "paper_2410_21149_amd", "covox.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    for kw in [dict(voxel_size=-1.0), dict(trunc_vox=0), dict(d_max=10.0), dict(precision=7), dict(n_min=0),
               dict(align_dof=5), dict(weight_mode=2), dict(integrator=2), dict(ray_carve=3),
               dict(integrator=1, precision=1)]:
        p = mod.default_params(**kw)
        h = ctypes.c_void_p()
        assert mod._lib.covox_create(ctypes.byref(h), ctypes.byref(p)) == mod.EINVAL


def test_struct_layouts_match_header():
    """ctypes mirrors of the public structs have the sizes the C compiler
    gives them (checked by compiling the header with gcc)."""
    import subprocess
    import tempfile
    src = r'''
#include <stdio.h>
#include "covox.h"
int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu ", sizeof(covox_params), sizeof(covox_align_stats),
 sizeof(covox_pair), sizeof(covox_submap_info), sizeof(covox_timing), sizeof(covox_summary_req),
 sizeof(covox_train_cfg), sizeof(covox_tuning));
 printf("%zu %zu %zu\n", sizeof(covox_pose_factor), sizeof(covox_pgo_cfg), sizeof(covox_pgo_stats));return 0;}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        sizes = [int(x) for x in subprocess.check_output([exe]).split()]
    import importlib.util
    spec = importlib.util.spec_from_file_location("_b3", os.path.join(ROOT, "paper_2410_21149_amd", "covox.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    assert sizes == [ctypes.sizeof(mod.covox_params), ctypes.sizeof(mod.covox_align_stats),
                     ctypes.sizeof(mod.covox_pair), ctypes.sizeof(mod.covox_submap_info),
                     ctypes.sizeof(mod.covox_timing), ctypes.sizeof(mod.covox_summary_req),
                     ctypes.sizeof(mod.covox_train_cfg), ctypes.sizeof(mod.covox_tuning),
                     ctypes.sizeof(mod.covox_pose_factor), ctypes.sizeof(mod.covox_pgo_cfg),
                     ctypes.sizeof(mod.covox_pgo_stats)]

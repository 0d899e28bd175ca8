"""Host-side checks of the C ABI (no GPU needed): the shared library loads and
exports every function include/lbm.h declares, and argument validation that
happens before any device call reports LBM_ERR_INVALID."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_1710_02375_amd import lbm

    if not os.path.exists(lbm.LIB_PATH):
        from paper_1710_02375_amd import build

        build.build()
    return lbm.LIB_PATH


def test_header_declares_the_core_abi():
    names = declared_functions()
    for core in ("lbm_create", "lbm_set_geometry", "lbm_step", "lbm_moments", "lbm_wall_force"):
        assert core in names


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (lbm_[a-z_]+)\b", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    lib = C.CDLL(libpath)
    for n in declared_functions():
        assert hasattr(lib, n)


def test_binding_names_match_header(libpath):
    from paper_1710_02375_amd import lbm

    assert set(lbm.EXPORTED) == set(declared_functions())


def test_invalid_descriptions_rejected_before_device_use(libpath):
    from paper_1710_02375_amd import lbm

    bad = [
        dict(Q=27, nx=8, ny=8, nz=8, nu=0.0),                      # nu <= 0
        dict(Q=9, nx=8, ny=8, nz=2, nu=0.1),                       # nz != 1 in 2D
        dict(Q=27, nx=0, ny=8, nz=8, nu=0.1),                      # empty axis
        dict(Q=27, nx=8, ny=8, nz=8, nu=0.1, storage=7),           # unknown storage
        dict(Q=27, nx=8, ny=8, nz=8, nu=0.1,                       # unpaired periodic face
             faces=["periodic", "wall", "periodic", "periodic", "periodic", "periodic"]),
        dict(Q=27, nx=8, ny=8, nz=8, nu=0.1,                       # inlet on +x
             faces=["wall", "inlet", "periodic", "periodic", "periodic", "periodic"]),
    ]
    for d in bad:
        with pytest.raises(lbm.LBMError) as ei:
            lbm.lbm_create([lbm.make_desc(**d)])
        assert ei.value.status == lbm.LBM_ERR_INVALID, d
    # mixed lattices in one context
    with pytest.raises(lbm.LBMError):
        lbm.lbm_create([lbm.make_desc(27, 8, 8, 8, 0.1), lbm.make_desc(9, 8, 8, 1, 0.1)])


def test_status_strings(libpath):
    from paper_1710_02375_amd import lbm

    for s in (0, -1, -2, -3, -4, -5, -6):
        assert lbm.lbm_status_string(s)

"""CPU checks of the C ABI: the library loads, exports every function that
include/dmwf.h declares, reports its ABI version, and refuses to create a
plan when no GPU is present (no compute call is made here)."""

import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmwf.h")
LIB = os.path.join(ROOT, "paper_1801_05358_amd", "libdmwf.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dm_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libdmwf.so is not built: run `python -m paper_1801_05358_amd.build`")
    from paper_1801_05358_amd import dmwf
    return dmwf.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("dm_plan_create", "dm_wiener_filter", "dm_wiener_filter_device", "dm_constrained_realizations",
              "dm_alm2map", "dm_map2alm", "dm_alm2map_adjoint", "dm_set_noise", "dm_set_spectra",
              "dm_set_schedule", "dm_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_1801_05358_amd import dmwf
    assert sorted(dmwf.exported_symbols()) == declared_functions()


def test_abi_version(lib):
    lib.dm_abi_version.restype = ctypes.c_int
    assert lib.dm_abi_version() == 11
    from paper_1801_05358_amd import dmwf
    header = open(HEADER).read()
    assert f"#define DMWF_ABI_VERSION {dmwf.ABI_VERSION}\n" in header
    assert dmwf.lib().dm_abi_version() == dmwf.ABI_VERSION


def test_no_device_is_reported_cleanly(lib):
    from paper_1801_05358_amd import dmwf
    if dmwf.device_count() > 0:
        pytest.skip("a GPU is present; covered by the gpu tests")
    with pytest.raises(dmwf.DmwfError) as e:
        dmwf.Plan(lmax=8, nside=4)
    assert e.value.status == dmwf.DM_EDEVICE


def test_null_plan_is_rejected(lib):
    from paper_1801_05358_amd import dmwf
    L = dmwf.lib()
    assert L.dm_plan_destroy(None) == dmwf.DM_EINVAL
    assert L.dm_set_schedule(None, None) == dmwf.DM_EINVAL
    assert L.dm_last_error(None) is not None


def test_product_path_has_no_cpu_fallback():
    """The binding and the library sources never import or call the oracle."""
    pkg = os.path.join(ROOT, "paper_1801_05358_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f


_RUNTIMES = """
import sys
sys.path.insert(0, {root!r})
from paper_1801_05358_amd import dmwf
dmwf.lib()
import torch
print(len(dmwf.hip_runtimes()), dmwf.hip_runtimes())
"""


def test_one_hip_runtime_when_the_binding_loads_first():
    """Loading the binding before torch must leave one HIP runtime mapped:
    torch's own copy, which the library's libamdhip64.so.7 resolves to."""
    r = subprocess.run([sys.executable, "-c", _RUNTIMES.format(root=ROOT)], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr
    n = int(r.stdout.split()[0])
    assert n == 1, r.stdout


_TWO = """
import ctypes, sys
sys.path.insert(0, {root!r})
ctypes.CDLL({lib!r})          # the library's own runtime first, bypassing the binding
from paper_1801_05358_amd import dmwf
try:
    dmwf.lib()
except RuntimeError as e:
    print("refused", e)
else:
    print("loaded", dmwf.hip_runtimes())
"""


def test_binding_refuses_two_hip_runtimes():
    r = subprocess.run([sys.executable, "-c", _TWO.format(root=ROOT, lib=LIB)], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("refused") and "two HIP runtimes" in r.stdout, r.stdout


def test_environment_variables_are_documented():
    """Every DMWF_* variable the library reads is listed in the header's
    account of plan creation, and nothing listed there is unread."""
    csrc = os.path.join(ROOT, "paper_1801_05358_amd", "csrc")
    read = set()
    for f in os.listdir(csrc):
        if f.endswith((".cpp", ".hip", ".h")):
            txt = open(os.path.join(csrc, f)).read()
            read |= set(re.findall(r'(?:env_int|getenv)\("(DMWF_[A-Z0-9_]+)"', txt))
    header = open(HEADER).read()
    listed = set(re.findall(r"^ \*\s+(DMWF_[A-Z0-9_]+)", header, flags=re.M))
    listed |= set(re.findall(r",\s+(DMWF_[A-Z0-9_]+)", " ".join(
        l for l in header.splitlines() if l.startswith(" *   DMWF_"))))
    assert read, "no environment reads found"
    assert read <= listed, f"read but not documented: {sorted(read - listed)}"
    assert listed <= read, f"documented but not read: {sorted(listed - read)}"

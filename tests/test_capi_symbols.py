"""The C-ABI library loads and exports every entry point include/*.h declares
(skei_ct.h: the CT operators; skei_mri.h: the multicoil MRI operator).

No compute call is made here (this runs without a GPU)."""
import ctypes
import glob
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


def declared():
    text = "\n".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(skei_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_expected_boundary():
    names = declared()
    for must in ("skei_geom_create", "skei_radon_fwd", "skei_radon_adj", "skei_radon_resid", "skei_fbp", "skei_fbp_adj",
                 "skei_rotate", "skei_rotate_adj", "skei_ei_loss_grad", "skei_strerror", "skei_mri_fwd",
                 "skei_mri_adj", "skei_coil_mix", "skei_coil_covariance", "skei_coil_pca"):
        assert must in names


def test_library_exports_every_declared_symbol(hiplib):
    out = subprocess.run(["nm", "-D", "--defined-only", hiplib], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (skei_\w+)$", out, flags=re.M))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binding_covers_header(hiplib):
    lib = ctypes.CDLL(hiplib)
    for name in declared():
        assert hasattr(lib, name)
    from paper_2411_05771_amd import capi
    assert sorted(capi.exported_symbols()) == declared()
    assert capi.version().startswith("skei_ct")
    assert "workspace" in capi.strerror(-5)

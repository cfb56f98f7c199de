"""Host-side checks of the C-ABI library that need no GPU: the shared library
loads and exports every function ``include/mcinv.h`` declares, and the
binding's signatures cover exactly those names."""

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcinv.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcinv_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for n in ("mcinv_create", "mcinv_load_csr", "mcinv_set_requested", "mcinv_burn_in", "mcinv_sample",
              "mcinv_read_estimates", "mcinv_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_cs_0412107_amd as pkg
    L = pkg.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", pkg._binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (mcinv_\w+)", out))
    assert set(_declared()) <= exported
    # and nothing else with C linkage: every unmangled global function is declared
    unmangled = {m for m in re.findall(r"\bT (\w+)", out) if not m.startswith("_")}
    assert unmangled == set(_declared()), sorted(unmangled ^ set(_declared()))


def test_binding_covers_header():
    from paper_cs_0412107_amd import _binding
    assert sorted(_binding.SIGNATURES) == _declared()


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_cs_0412107_amd as pkg
    with pytest.raises(pkg.McinvError) as ei:
        pkg.mcinv_create(n_pairs=4)
    assert ei.value.code in (pkg.MCINV_EDEVICE,)


def test_bad_config_rejected_before_device():
    import paper_cs_0412107_amd as pkg
    with pytest.raises(pkg.McinvError) as ei:
        pkg.mcinv_create(n_pairs=12, n_groups=2)   # 6 pairs per group
    assert ei.value.code == pkg.MCINV_EINVAL
    with pytest.raises(pkg.McinvError) as ei:
        pkg.mcinv_create(n_pairs=8, n_groups=3)
    assert ei.value.code == pkg.MCINV_EINVAL

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


def test_binding_constants_match_header():
    from paper_cs_0412107_amd import _binding
    text = open(HEADER).read()
    defs = re.findall(r"#define (MCINV_\w+)\s+\(?(-?\d+)u?\)?", text)
    assert len(defs) > 20
    for name, value in defs:
        assert getattr(_binding, name) == int(value), name


def test_every_entry_point_catches_exceptions():
    """No C++ exception may leave the library: each exported function that
    returns a status is a function-try-block whose handler converts the
    exception into a status."""
    csrc = os.path.join(ROOT, "paper_cs_0412107_amd", "csrc")
    found = {}
    for fn in sorted(os.listdir(csrc)):
        if not fn.endswith(".hip"):
            continue
        lines = open(os.path.join(csrc, fn)).read().split("\n")
        for i, line in enumerate(lines):
            m = re.match(r'^(?:extern "C" )?mcinv_status (mcinv_\w+)\(', line)
            if not m:
                continue
            j = i
            while lines[j] not in ("{", "try {"):
                j += 1
            k = j
            while lines[k] != "}":
                k += 1
            found[m.group(1)] = (lines[j] == "try {" and lines[k - 2] == "} catch (...) {"
                                 and "exception_status" in lines[k - 1])
    status_fns = [n for n in _declared() if re.search(r"mcinv_status\s+" + n + r"\s*\(", open(HEADER).read())]
    assert sorted(found) == sorted(status_fns)
    assert all(found.values()), [n for n, ok in found.items() if not ok]


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


def _csr(n, rows):
    """CSR arrays from per-row (column, value) lists, kept in the given order."""
    import numpy as np
    rp = [0]
    col, val = [], []
    for r in rows:
        col += [c for c, _ in r]
        val += [v for _, v in r]
        rp.append(len(col))
    return (n, len(col), np.array(rp, dtype=np.int64), np.array(col, dtype=np.int32),
            np.array(val, dtype=np.float64))


@pytest.mark.parametrize("case,code,text", [
    ("unsorted", "EINVAL", "strictly increasing"),
    ("duplicate", "EINVAL", "strictly increasing"),
    ("range", "EINVAL", "out of range"),
    ("no_diag", "ESINGULAR", "row 2 has no nonzero diagonal"),
    ("zero_diag", "ESINGULAR", "row 1 has no nonzero diagonal"),
    ("both", "EINVAL", "out of range"),          # a pattern error outranks a missing diagonal
    ("row_ptr", "EINVAL", "row_ptr is decreasing"),
])
def test_csr_validation_on_the_host(case, code, text):
    """The host preparation's CSR checks (run before any device call, here
    through mcinv_features): the error code and the reported row."""
    import paper_cs_0412107_amd as pkg
    good = [[(0, 4.0), (1, 1.0)], [(0, 1.0), (1, 4.0), (3, 1.0)], [(1, 1.0), (2, 4.0)], [(2, 1.0), (3, 4.0)]]
    rows = [list(r) for r in good]
    if case == "unsorted":
        rows[1] = [(1, 4.0), (0, 1.0), (3, 1.0)]
    elif case == "duplicate":
        rows[3] = [(3, 4.0), (3, 1.0)]
    elif case == "range":
        rows[2] = [(1, 1.0), (2, 4.0), (7, 1.0)]
    elif case == "no_diag":
        rows[2] = [(1, 1.0)]
    elif case == "zero_diag":
        rows[1] = [(0, 1.0), (1, 0.0), (3, 1.0)]
    elif case == "both":
        rows[1] = [(0, 1.0), (3, 1.0)]               # row 1 lacks its diagonal ...
        rows[3] = [(3, 4.0), (9, 1.0)]               # ... and row 3 has a column out of range
    n, nnz, rp, col, val = _csr(4, rows)
    if case == "row_ptr":
        rp = rp.copy()
        rp[2], rp[3] = rp[3], rp[2]
    with pytest.raises(pkg.McinvError) as ei:
        pkg.mcinv_features(0, n, nnz, rp, col, val)
    assert ei.value.code == getattr(pkg, "MCINV_" + code), (ei.value.code, str(ei.value))
    assert text in str(ei.value), str(ei.value)


def test_valid_csr_passes_the_host_checks():
    import torch
    import paper_cs_0412107_amd as pkg
    good = [[(0, 4.0), (1, 1.0)], [(0, 1.0), (1, 4.0), (3, 1.0)], [(1, 1.0), (2, 4.0)], [(2, 1.0), (3, 4.0)]]
    n, nnz, rp, col, val = _csr(4, good)
    if torch.cuda.is_available():
        assert pkg.mcinv_features(0, n, nnz, rp, col, val).shape == (4, 32)
    else:
        with pytest.raises(pkg.McinvError) as ei:   # validated, then no device
            pkg.mcinv_features(0, n, nnz, rp, col, val)
        assert ei.value.code == pkg.MCINV_EDEVICE


def test_bench_refuses_several_gpus():
    """The benchmark runs on one GPU; asking for more exits with a message."""
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr, (r.returncode, r.stderr[-300:])

"""The allocation-free features entry point (mcinv_features_noalloc) against
mcinv_features through the C-ABI: the same kernels on the caller's device
arrays with the library's fixed scratch array, so the features must be equal
bit for bit -- on two calls in a row, the second with a smaller matrix (the
scratch keeps the first call's contents), and again after refused calls."""

import numpy as np
import pytest

import gen
from gpu_util import print_case

pytestmark = pytest.mark.gpu

mc = pytest.importorskip("paper_cs_0412107_amd")
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _device_csr(m):
    rp = torch.tensor(np.asarray(m.row_ptr, dtype=np.int64), device="cuda")
    col = torch.tensor(np.asarray(m.col, dtype=np.int32), device="cuda")
    val = torch.tensor(np.asarray(m.val, dtype=np.float64), device="cuda")
    return rp, col, val


def _noalloc(m, rp=None, col=None, val=None):
    if rp is None:
        rp, col, val = _device_csr(m)
    out = torch.full((m.n, mc.MCINV_N_FEATURES), float("nan"), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    mc.mcinv_features_noalloc(0, m.n, m.nnz, rp.data_ptr(), col.data_ptr(), val.data_ptr(), out.data_ptr(),
                              stream)
    return out.cpu().numpy()


def _params(k):
    q = gen.surrogate_params(k + 1, seed=4040)[k]
    return q


def test_noalloc_equals_features_two_calls():
    q = _params(0)
    big = gen.pedigree(20000, seed=q["seed"], founders=q["founders"], lam=q["lam"], factor=q["factor"])
    small = gen.pedigree(1500, seed=77)
    for m in (big, small):                       # the second call is smaller than the first
        print_case(test="noalloc", n=m.n, nnz=m.nnz)
        ref = mc.mcinv_features(0, m.n, m.nnz, m.row_ptr, m.col, m.val)
        got = _noalloc(m)
        assert np.array_equal(got, ref)


def test_noalloc_at_its_size_limits_and_refusals():
    mats = [gen.random_dominant(32768, 7, seed=5), gen.random_dominant(300, 4, seed=6)]
    assert mats[0].nnz == 262144
    for m in mats:
        print_case(test="noalloc_limit", n=m.n, nnz=m.nnz)
        ref = mc.mcinv_features(0, m.n, m.nnz, m.row_ptr, m.col, m.val)
        assert np.array_equal(_noalloc(m), ref)
    m = mats[1]
    rp, col, val = _device_csr(m)
    out = torch.empty((m.n, mc.MCINV_N_FEATURES), dtype=torch.float32, device="cuda")
    # sizes beyond the scratch array: refused before any device work
    for n, nnz in ((32769, 32769), (300, 262145), (0, 0)):
        with pytest.raises(mc.McinvError) as ei:
            mc.mcinv_features_noalloc(0, n, nnz, rp.data_ptr(), col.data_ptr(), val.data_ptr(), out.data_ptr())
        assert ei.value.code == mc.MCINV_EINVAL
    # a zero diagonal: ESINGULAR; columns out of order: EINVAL (checked on the device)
    d = np.asarray(m.val).copy()
    rows = np.repeat(np.arange(m.n), np.diff(m.row_ptr))
    d[np.nonzero(np.asarray(m.col) == rows)[0][17]] = 0.0
    with pytest.raises(mc.McinvError) as ei:
        _noalloc(m, rp, col, torch.tensor(d, device="cuda"))
    assert ei.value.code == mc.MCINV_ESINGULAR
    c = np.asarray(m.col).copy()
    b = int(m.row_ptr[40])
    c[b], c[b + 1] = c[b + 1], c[b]
    with pytest.raises(mc.McinvError) as ei:
        _noalloc(m, rp, torch.tensor(c, device="cuda"), val)
    assert ei.value.code == mc.MCINV_EINVAL
    # and a valid call after the refusals
    ref = mc.mcinv_features(0, m.n, m.nnz, m.row_ptr, m.col, m.val)
    assert np.array_equal(_noalloc(m, rp, col, val), ref)

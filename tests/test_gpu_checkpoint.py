"""Checkpoint / resume through the C-ABI: a context restored from a file
continues bit for bit as the saved one (states, every estimate and standard
error), in both moment layouts (chain groups and time batches), in hermitian
mode and with a Q trace; mismatched configurations and damaged files are
rejected."""

import os

import numpy as np
import pytest
import scipy.sparse as sp

import gen
from gpu_util import oracle_matrix, print_case

pytestmark = pytest.mark.gpu

mc = pytest.importorskip("paper_cs_0412107_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _estimates(s, with_q):
    out = [s.diag(), s.trace(), s.block(), s.entries(), (s.state(0), s.state(1))]
    if with_q:
        out.append(s.qtrace())
    return out


def _same(a, b):
    for x, y in zip(a, b):
        for u, v in zip(x, y):
            assert np.array_equal(np.asarray(u), np.asarray(v), equal_nan=True)


@pytest.mark.parametrize("dtype,G,herm", [("f32", 16, False), ("f64", 1, False), ("c64", 4, False),
                                          ("f32", 16, True)])
def test_resume_is_bit_identical(tmp_path, dtype, G, herm):
    print_case(test="checkpoint", dtype=dtype, G=G, herm=herm)
    if dtype == "c64":
        m = gen.lattice(6, k=0.12, seed=91)
    elif herm:
        m = gen.pedigree(1500, seed=92, lam=0.0, symmetric=True)
    else:
        m = gen.pedigree(1500, seed=92)
    m = oracle_matrix(m, dtype)
    rows = np.array([3, 7, 100, 999])
    ent = [(0, 1), (5, 5), (77, 3)]
    Q = sp.random(m.n, m.n, density=3.0 / m.n, random_state=np.random.default_rng(1), format="csr") + \
        sp.identity(m.n)
    path = str(tmp_path / "ck.bin")

    def make():
        s = mc.Sampler(m, pairs=64, groups=G, dtype=dtype, seed=123, hermitian=herm)
        s.set_trace_matrix(Q)
        s.request(diag=True, trace=True, block_rows=rows, block_cols=rows[::-1], entries=ent, qtrace=True)
        return s

    with make() as a:
        a.burn_in(4)
        a.request(diag=True, trace=True, block_rows=rows, block_cols=rows[::-1], entries=ent, qtrace=True)
        a.sample(37)          # time batches merge along the way when G < 16
        a.save(path)
        a.sample(29)
        ref = _estimates(a, True)
        info_a = a.info()
    with make() as b:
        b.restore(path)
        b.sample(29)
        got = _estimates(b, True)
        info_b = b.info()
    _same(got, ref)
    for k in ("sweeps_done", "samples_done", "batch_len", "n_batches"):
        assert info_a[k] == info_b[k], k


def test_restore_rejects_mismatch(tmp_path):
    m = oracle_matrix(gen.pedigree(800, seed=93), "f32")
    path = str(tmp_path / "ck.bin")
    with mc.Sampler(m, pairs=32, dtype="f32", seed=1) as a:
        a.burn_in(2)
        a.save(path)
    for kw in ({"seed": 2}, {"pairs": 64}):
        args = dict(pairs=32, dtype="f32", seed=1)
        args.update(kw)
        with mc.Sampler(m, **args) as b:
            with pytest.raises(mc.McinvError) as ei:
                b.restore(path)
            assert ei.value.code == mc.MCINV_EINVAL
    with mc.Sampler(oracle_matrix(gen.pedigree(800, seed=94), "f32"), pairs=32, dtype="f32", seed=1) as b:
        with pytest.raises(mc.McinvError) as ei:
            b.restore(path)
        assert ei.value.code == mc.MCINV_EINVAL
    with open(path, "rb") as f:
        data = f.read()
    cut = str(tmp_path / "cut.bin")
    with open(cut, "wb") as f:
        f.write(data[: len(data) // 2])
    with mc.Sampler(m, pairs=32, dtype="f32", seed=1) as b:
        with pytest.raises(mc.McinvError) as ei:
            b.restore(cut)
        assert ei.value.code == mc.MCINV_EINVAL
        with pytest.raises(mc.McinvError):
            b.restore(os.path.join(str(tmp_path), "missing.bin"))
        b.restore(path)
        assert b.info()["sweeps_done"] == 2


def test_restore_rejects_corrupt_counts(tmp_path):
    """Counts read from a checkpoint header (index lists, samples) are checked
    against the bytes left in the file before they size any buffer: a damaged
    header is EINVAL, not a huge allocation, and the context stays usable."""
    import struct
    print_case(test="checkpoint_corrupt_counts")
    m = oracle_matrix(gen.pedigree(600, seed=95), "f32")
    rows = np.array([1, 2, 3])
    path = str(tmp_path / "ck.bin")
    # header: 8 magic bytes, then 64-bit fields in declaration order
    fields = ["version", "n", "nnz", "n_off", "P", "ld", "G", "dtype", "hermitian", "noise", "stream_id", "seed",
              "fingerprint", "flags", "nI", "nJ", "ne", "sweeps", "samples", "batch_len", "nslots", "q_nnz",
              "requested", "pair_offset"]
    off = {f: 8 + 8 * i for i, f in enumerate(fields)}
    with mc.Sampler(m, pairs=64, groups=16, dtype="f32", seed=3) as a:
        a.burn_in(2)
        a.request(diag=True, trace=True, block_rows=rows, block_cols=rows, entries=[(0, 1)])
        a.sample(5)
        a.save(path)
        ref = a.diag()
    data = open(path, "rb").read()
    assert struct.unpack_from("<q", data, off["nI"])[0] == 3
    assert struct.unpack_from("<q", data, off["samples"])[0] == 5
    bad = str(tmp_path / "bad.bin")
    with mc.Sampler(m, pairs=64, groups=16, dtype="f32", seed=3) as b:
        for field, value in (("nI", 1 << 40), ("nJ", -1), ("ne", 1 << 40), ("ne", -2), ("samples", 1 << 40),
                             ("samples", -5), ("samples", 99)):
            d = bytearray(data)
            struct.pack_into("<q", d, off[field], value)
            open(bad, "wb").write(bytes(d))
            with pytest.raises(mc.McinvError) as ei:
                b.restore(bad)
            assert ei.value.code == mc.MCINV_EINVAL, (field, value)
        for cut in (len(data) - 8, len(data) - 1):     # truncated, and one byte short
            open(bad, "wb").write(data[:cut])
            with pytest.raises(mc.McinvError) as ei:
                b.restore(bad)
            assert ei.value.code == mc.MCINV_EINVAL
        open(bad, "wb").write(data + b"\0" * 8)          # trailing bytes
        with pytest.raises(mc.McinvError) as ei:
            b.restore(bad)
        assert ei.value.code == mc.MCINV_EINVAL
        assert b.info()["sweeps_done"] == 0              # none of the failed restores changed the context
        b.restore(path)
        got = b.diag()
    for x, y in zip(got, ref):
        assert np.array_equal(np.asarray(x), np.asarray(y))


def test_restore_rejects_same_pattern_other_values(tmp_path):
    """The fingerprint covers the matrix values, not only its pattern: a
    checkpoint does not restore onto a matrix with the same pattern and other
    values (its chains and sums belong to the first matrix), nor, when the Q
    trace is accumulated, onto another Q with the same pattern."""
    import scipy.sparse as sp
    print_case(test="checkpoint_values")
    m = oracle_matrix(gen.pedigree(700, seed=96), "f32")
    other = gen.CSR(n=m.n, row_ptr=m.row_ptr.copy(), col=m.col.copy(), val=m.val.copy())
    k = int(np.nonzero(other.col != np.repeat(np.arange(m.n), np.diff(m.row_ptr)))[0][0])
    other.val[k] *= 0.5                        # one off-diagonal value changed
    Q = sp.random(m.n, m.n, density=3.0 / m.n, random_state=np.random.default_rng(5), format="csr") + \
        sp.identity(m.n)
    Q2 = Q.copy()
    Q2.data[0] += 1.0
    path = str(tmp_path / "ck.bin")
    pathq = str(tmp_path / "ckq.bin")
    with mc.Sampler(m, pairs=32, dtype="f32", seed=4) as a:
        a.burn_in(2)
        a.save(path)
        a.set_trace_matrix(Q)
        a.request(diag=True, trace=True, qtrace=True)
        a.sample(3)
        a.save(pathq)
    with mc.Sampler(other, pairs=32, dtype="f32", seed=4) as b:
        with pytest.raises(mc.McinvError) as ei:
            b.restore(path)
        assert ei.value.code == mc.MCINV_EINVAL
        assert b.info()["sweeps_done"] == 0
    with mc.Sampler(m, pairs=32, dtype="f32", seed=4) as b:
        b.restore(path)                         # the same matrix restores
        assert b.info()["sweeps_done"] == 2
        b.set_trace_matrix(Q2)
        with pytest.raises(mc.McinvError) as ei:
            b.restore(pathq)
        assert ei.value.code == mc.MCINV_EINVAL
        b.set_trace_matrix(Q)
        b.restore(pathq)
        assert b.info()["samples_done"] == 3

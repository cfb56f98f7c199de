"""CPU oracle for the correlated-chains Monte Carlo inverter.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check
and by the benchmark's CPU-baseline leg, never by the GPU library.  The sweep
itself is plain C (``mcinv_oracle.c``, complex128 arithmetic, one thread);
this module marshals arguments and finalizes estimates with NumPy.

Paper: Garcia-Cortes & Cabrillo, "A Monte Carlo algorithm for efficient large
matrix inversion".  Equation names follow the paper's labels.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import theory  # noqa: F401  (dense closed forms used by the pins)
from .estimators import cluster_estimate, geyer_ips  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcinv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The same source optimised for the host (AVX2/FMA-level x86-64, contraction of
# a*b+c into fused operations off, so the arithmetic is unchanged): the build
# the benchmark times as the CPU baseline.  The tests use the plain build.
_LIB_FAST = os.path.join(_HERE, "liboracle_fast.so")
FAST_FLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off"]

NOISE_NORMAL = 0
NOISE_RADEMACHER = 1
NOISE_NONE = 2


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, IEEE semantics kept), and the same
    source with FAST_FLAGS for the benchmark's CPU baseline."""
    for path, flags in ((_LIB, ["-O2"]), (_LIB_FAST, FAST_FLAGS)):
        if force or not os.path.exists(path):
            tmp = path + ".tmp"
            subprocess.check_call(["gcc", *flags, "-std=c11", "-fPIC", "-shared", "-Wall",
                                   "-o", tmp, _SRC, "-lm"])
            os.replace(tmp, path)
    return _LIB


class _Moments(ctypes.Structure):
    _fields_ = [
        ("groups", ctypes.c_int64),
        ("pairs_total", ctypes.c_int64),
        ("batch_len", ctypes.c_int64),
        ("n_batches", ctypes.c_int64),
        ("samples_done", ctypes.c_int64),
        ("want_diag", ctypes.c_int32),
        ("pad_", ctypes.c_int32),
        ("diag", ctypes.c_void_p),
        ("nI", ctypes.c_int64),
        ("nJ", ctypes.c_int64),
        ("bI", ctypes.c_void_p),
        ("bJ", ctypes.c_void_p),
        ("block", ctypes.c_void_p),
        ("n_entries", ctypes.c_int64),
        ("ei", ctypes.c_void_p),
        ("ej", ctypes.c_void_p),
        ("entries", ctypes.c_void_p),
        ("trace_series", ctypes.c_void_p),
        ("max_samples", ctypes.c_int64),
        ("cluster_count", ctypes.c_void_p),
    ]


_libs = {}


def lib(fast=False):
    """The plain build, or with ``fast`` the FAST_FLAGS build (same source)."""
    if fast not in _libs:
        path = _LIB_FAST if fast else _LIB
        if not os.path.exists(path):
            build(force=False)
        L = ctypes.CDLL(path)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        u32 = ctypes.c_uint32
        u64 = ctypes.c_uint64
        L.ora_philox4x32_10.argtypes = [p, p, p]
        L.ora_philox4x32_10.restype = None
        L.ora_noise_block.argtypes = [u64, u32, u32, u32, u32, ctypes.c_int, p]
        L.ora_noise_block.restype = None
        L.ora_noise.argtypes = [u64, u32, i64, i64, i64, ctypes.c_int]
        L.ora_noise.restype = ctypes.c_double
        L.ora_greedy_color.argtypes = [i64, p, p, p, p, p]
        L.ora_greedy_color.restype = ctypes.c_int
        L.ora_sweeps.argtypes = [i64, p, p, p, ctypes.c_int, p, u64, u32, ctypes.c_int,
                                 i64, p, p, p, i64, i64, ctypes.POINTER(_Moments)]
        L.ora_sweeps.restype = ctypes.c_int
        _libs[fast] = L
    return _libs[fast]


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ora_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def noise(seed, stream, rows, sweeps, pairs, kind=NOISE_NORMAL):
    """phi(row, sweep, pair) for broadcast index arrays (one C call each)."""
    r, k, p = np.broadcast_arrays(np.asarray(rows), np.asarray(sweeps), np.asarray(pairs))
    out = np.empty(r.shape, dtype=np.float64)
    f = lib().ora_noise
    for idx in np.ndindex(r.shape):
        out[idx] = f(seed, stream, int(r[idx]), int(k[idx]), int(p[idx]), kind)
    return out


def greedy_color(m):
    """Greedy multicolouring; returns (color int32[n], order int64[n], ncolors)."""
    color = np.zeros(m.n, dtype=np.int32)
    order = np.zeros(m.n, dtype=np.int64)
    nc = ctypes.c_int32(0)
    rp = np.ascontiguousarray(m.row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(m.col, dtype=np.int32)
    lib().ora_greedy_color(m.n, _ptr(rp), _ptr(ci), _ptr(color), _ptr(order),
                           ctypes.byref(nc))
    return color, order, int(nc.value)


class OracleError(RuntimeError):
    pass


def coupled_burn_in(m, seed, tol, max_sweeps, order=None, stream=0, noise_kind=NOISE_NORMAL, pair_ids=(0,)):
    """Algorithm 1, steps 1-5, literally: paths started at z = w = 0 and at
    z* = w* = i (1-based index), driven by the same noise, swept together
    until max_i |z_i - z*_i| < tol and max_i |w_i - w*_i| < tol.  Returns the
    number of sweeps N and the differences after each sweep."""
    if order is None:
        _, order, _ = greedy_color(m)
    a = Run(m, seed, pairs=len(pair_ids), pair_ids=pair_ids, order=order, stream=stream, noise_kind=noise_kind)
    b = Run(m, seed, pairs=len(pair_ids), pair_ids=pair_ids, order=order, stream=stream, noise_kind=noise_kind)
    start = np.arange(1, m.n + 1, dtype=np.float64)[:, None]
    b.z[:] = start
    b.w[:] = start
    diffs = []
    for k in range(1, max_sweeps + 1):
        a.burn_in(1)
        b.burn_in(1)
        dz = float(np.max(np.abs(b.z - a.z)))
        dw = float(np.max(np.abs(b.w - a.w)))
        diffs.append((dz, dw))
        if dz < tol and dw < tol:
            return k, diffs
    return max_sweeps, diffs


class Run:
    """One oracle run: ``pairs`` chain pairs (global ids ``pair_ids``) of the
    correlated-chains sampler on matrix ``m``.

    State ``z``, ``w`` is complex128 [n][len(pair_ids)] in original row order.
    ``order`` is the sweep order (default: the greedy multicolour order).
    """

    def __init__(self, m, seed, pairs, groups=1, pair_ids=None, order=None, stream=0,
                 noise_kind=NOISE_NORMAL, n_batches_max=64, fast=False):
        self.m = m
        self.fast = bool(fast)
        self.n = m.n
        self.seed = int(seed)
        self.stream = int(stream)
        self.noise_kind = int(noise_kind)
        self.pairs_total = int(pairs)
        self.groups = int(groups)
        if self.pairs_total % self.groups:
            raise ValueError("pairs must be a multiple of groups")
        self.pair_ids = np.arange(pairs, dtype=np.int64) if pair_ids is None else \
            np.ascontiguousarray(pair_ids, dtype=np.int64)
        if order is None:
            _, order, _ = greedy_color(m)
        self.order = np.ascontiguousarray(order, dtype=np.int64)
        self.z = np.zeros((self.n, self.pair_ids.size), dtype=np.complex128)
        self.w = np.zeros_like(self.z)
        self.sweeps_done = 0
        self.n_batches_max = n_batches_max
        self._rp = np.ascontiguousarray(m.row_ptr, dtype=np.int64)
        self._ci = np.ascontiguousarray(m.col, dtype=np.int32)
        if m.is_complex:
            self._val = np.ascontiguousarray(m.val, dtype=np.complex128).view(np.float64)
        else:
            self._val = np.ascontiguousarray(m.val, dtype=np.float64)
        self.mom = None

    # -- requested quantities -------------------------------------------------
    def request(self, samples, diag=True, block_rows=None, block_cols=None,
                entries=None, trace=True):
        """Allocate accumulators for ``samples`` sample sweeps.  Time batches:
        the smallest power-of-two batch length L with ceil(samples/L) <= 64
        when there are fewer than 16 groups, one batch otherwise."""
        G = self.groups
        if G >= 16:
            L, nb = max(1, samples), 1
        else:
            L = 1
            while -(-samples // L) > self.n_batches_max:
                L *= 2
            nb = -(-samples // L)
        self.batch_len, self.n_batches = L, nb
        self.samples_max = samples
        n = self.n
        self.diag_acc = np.zeros((nb, G, n), dtype=np.complex128) if diag else None
        self.I = np.ascontiguousarray(block_rows if block_rows is not None else [], dtype=np.int64)
        self.J = np.ascontiguousarray(block_cols if block_cols is not None else [], dtype=np.int64)
        self.block_acc = np.zeros((nb, G, self.I.size, self.J.size), dtype=np.complex128) \
            if self.I.size and self.J.size else None
        if entries is not None and len(entries):
            e = np.asarray(entries, dtype=np.int64).reshape(-1, 2)
            self.ei = np.ascontiguousarray(e[:, 0])
            self.ej = np.ascontiguousarray(e[:, 1])
            self.entry_acc = np.zeros((nb, G, e.shape[0]), dtype=np.complex128)
        else:
            self.ei = self.ej = np.zeros(0, dtype=np.int64)
            self.entry_acc = None
        self.series = np.zeros(samples, dtype=np.complex128) if trace else None
        self.counts = np.zeros((nb, G), dtype=np.float64)
        mo = _Moments()
        mo.groups = G
        mo.pairs_total = self.pairs_total
        mo.batch_len = L
        mo.n_batches = nb
        mo.samples_done = 0
        mo.want_diag = 1 if diag else 0
        mo.diag = _ptr(self.diag_acc)
        mo.nI = self.I.size if self.block_acc is not None else 0
        mo.nJ = self.J.size if self.block_acc is not None else 0
        mo.bI = _ptr(self.I)
        mo.bJ = _ptr(self.J)
        mo.block = _ptr(self.block_acc)
        mo.n_entries = self.ei.size
        mo.ei = _ptr(self.ei)
        mo.ej = _ptr(self.ej)
        mo.entries = _ptr(self.entry_acc)
        mo.trace_series = _ptr(self.series)
        mo.max_samples = samples
        mo.cluster_count = _ptr(self.counts)
        self.mom = mo

    # -- sweeps ---------------------------------------------------------------
    def _run(self, sweeps, accumulate):
        m = self.m
        st = lib(self.fast).ora_sweeps(
            m.n, _ptr(self._rp), _ptr(self._ci), _ptr(self._val), 1 if m.is_complex else 0,
            _ptr(self.order), self.seed, self.stream, self.noise_kind,
            self.pair_ids.size, _ptr(self.pair_ids),
            _ptr(self.z.view(np.float64)), _ptr(self.w.view(np.float64)),
            self.sweeps_done, sweeps, ctypes.byref(self.mom) if accumulate else None)
        if st == 2:
            raise OracleError("diverged")
        if st == 3:
            raise OracleError("zero or missing diagonal")
        if st != 0:
            raise OracleError(f"oracle status {st}")
        self.sweeps_done += sweeps

    def burn_in(self, sweeps):
        self._run(int(sweeps), False)

    def sample(self, sweeps):
        if self.mom is None:
            raise OracleError("request() first")
        if getattr(self, "Q", None) is None:
            self._run(int(sweeps), True)
            return
        for _ in range(int(sweeps)):
            self._run(1, True)
            # eq tr with a general Q: sum over the pairs of w^dagger Q z, after this sweep
            self.qseries.append(complex(np.sum(np.conj(self.w) * (self.Q @ self.z))))

    def set_trace_matrix(self, Q):
        """Q (scipy sparse, n x n) for tr(Q C^-1) = E[w^dagger Q z]; call before sample()."""
        self.Q = Q.tocsr().astype(np.complex128)
        self.qseries = []

    def qtrace(self):
        """tr(Q C^-1) estimate and Geyer standard error from the per-sweep series."""
        x = np.array(self.qseries, dtype=np.complex128) / self.pair_ids.size
        return geyer_ips(x)

    @property
    def samples_done(self):
        return 0 if self.mom is None else int(self.mom.samples_done)

    # -- finalize -------------------------------------------------------------
    def _clusters(self, acc):
        nb, G = acc.shape[:2]
        return acc.reshape((nb * G,) + acc.shape[2:]), self.counts.reshape(nb * G)

    def diag(self):
        s, c = self._clusters(self.diag_acc)
        return cluster_estimate(s, c)

    def block(self):
        s, c = self._clusters(self.block_acc)
        return cluster_estimate(s, c)

    def entries(self):
        s, c = self._clusters(self.entry_acc)
        return cluster_estimate(s, c)

    def trace(self):
        """Trace estimate (mean over samples of sum_i z_i conj(w_i), per pair)
        and its Geyer initial-positive-sequence standard error."""
        x = self.series[: self.samples_done] / self.pair_ids.size
        return geyer_ips(x)

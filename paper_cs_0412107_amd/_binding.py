"""ctypes binding of ``libmcinv.so`` (declared in ``include/mcinv.h``).

Every ``mcinv_*`` function here has the name and the argument order of the
C entry point; it converts NumPy arrays to pointers, raises
:class:`McinvError` on a negative status and returns outputs as arrays.  No
step of the method runs in Python.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmcinv.so")

MCINV_OK = 0
MCINV_EINVAL = -1
MCINV_ESINGULAR = -2
MCINV_ESTATE = -3
MCINV_ENOMEM = -4
MCINV_EDEVICE = -5
MCINV_EDIVERGED = -6
MCINV_EINTERNAL = -7

MCINV_R32, MCINV_R64, MCINV_C64, MCINV_C128 = 0, 1, 2, 3
MCINV_NOISE_NORMAL, MCINV_NOISE_RADEMACHER, MCINV_NOISE_NONE = 0, 1, 2
MCINV_MOMENTS_FP64, MCINV_MOMENTS_BF16X3 = 0, 1
MCINV_REQ_DIAG, MCINV_REQ_TRACE, MCINV_REQ_BLOCK, MCINV_REQ_ENTRIES = 1, 2, 4, 8
MCINV_REQ_QTRACE = 16

DTYPES = {"f32": MCINV_R32, "f64": MCINV_R64, "c64": MCINV_C64, "c128": MCINV_C128}
NP_STATE = {MCINV_R32: np.float32, MCINV_R64: np.float64, MCINV_C64: np.complex64,
            MCINV_C128: np.complex128}


class McinvError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"mcinv error {code}: {message}")
        self.code = code


class mcinv_config(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32),
        ("sweep_dtype", ctypes.c_int32),
        ("moments", ctypes.c_int32),
        ("noise", ctypes.c_int32),
        ("n_pairs", ctypes.c_int64),
        ("n_groups", ctypes.c_int32),
        ("stream_id", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("stream", ctypes.c_void_p),
        ("profile", ctypes.c_int32),
        ("pass_tiles", ctypes.c_int32),
        ("xcd_order", ctypes.c_int32),
        ("hermitian", ctypes.c_int32),
        ("pair_offset", ctypes.c_int64),
        ("stores", ctypes.c_int32),
    ]


class mcinv_info(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("n_pairs", ctypes.c_int64), ("ld", ctypes.c_int64),
        ("n_colors", ctypes.c_int32), ("n_groups", ctypes.c_int32),
        ("sweeps_done", ctypes.c_int64), ("samples_done", ctypes.c_int64),
        ("batch_len", ctypes.c_int64), ("n_batches", ctypes.c_int64),
        ("offdiag_entries", ctypes.c_int64),
        ("sweep_kernel_ms", ctypes.c_double), ("sweep_kernel_launches", ctypes.c_int64),
        ("moment_kernel_ms", ctypes.c_double), ("moment_kernel_launches", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class mcinv_batch_config(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32),
        ("noise", ctypes.c_int32),
        ("n_pairs", ctypes.c_int64),
        ("n_groups", ctypes.c_int32),
        ("rows_per_item", ctypes.c_int32),
        ("grab", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("stream", ctypes.c_void_p),
    ]


class mcinv_batch_info(ctypes.Structure):
    _fields_ = [
        ("n_matrices", ctypes.c_int64), ("n_rows", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("n_pairs", ctypes.c_int64),
        ("n_groups", ctypes.c_int32), ("max_colors", ctypes.c_int32), ("rows_per_item", ctypes.c_int32),
        ("grab", ctypes.c_int32), ("grid", ctypes.c_int32), ("schedule", ctypes.c_int32),
        ("items_per_sweep", ctypes.c_int64), ("sweeps_done", ctypes.c_int64), ("samples_done", ctypes.c_int64),
        ("last_call_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class mcinv_gate_config(ctypes.Structure):
    _fields_ = [("feature_a", ctypes.c_int32), ("feature_b", ctypes.c_int32), ("bins", ctypes.c_int32),
                ("min_rows", ctypes.c_int32), ("tol", ctypes.c_double), ("ucb_z", ctypes.c_double)]


_lib = None

# name -> (restype, argtypes)
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64
_D = ctypes.c_double
SIGNATURES = {
    "mcinv_create": (_I32, [ctypes.POINTER(mcinv_config), ctypes.POINTER(_P)]),
    "mcinv_destroy": (None, [_P]),
    "mcinv_load_csr": (_I32, [_P, _I64, _I64, _P, _P, _P, _I32]),
    "mcinv_set_requested": (_I32, [_P, _U32, _P, _I64, _P, _I64, _P, _P, _I64]),
    "mcinv_burn_in": (_I32, [_P, _I64]),
    "mcinv_burn_in_coupled": (_I32, [_P, _D, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "mcinv_sample": (_I32, [_P, _I64]),
    "mcinv_sample_until": (_I32, [_P, _D, _I64, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_D)]),
    "mcinv_sample_until_trace": (_I32, [_P, _D, _I64, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_D)]),
    "mcinv_read_trace_stats": (_I32, [_P, _U32, _P]),
    "mcinv_read_estimates": (_I32, [_P, _U32, _P, _P, _I64]),
    "mcinv_read_state": (_I32, [_P, _I32, _P, _I64]),
    "mcinv_write_state": (_I32, [_P, _I32, _P, _I64]),
    "mcinv_get_permutation": (_I32, [_P, _P, _P]),
    "mcinv_set_stop_rows": (_I32, [_P, _P, _I64]),
    "mcinv_set_trace_matrix": (_I32, [_P, _I64, _P, _P, _P, _I32]),
    "mcinv_save": (_I32, [_P, ctypes.c_char_p]),
    "mcinv_restore": (_I32, [_P, ctypes.c_char_p]),
    "mcinv_tune_launch": (_I32, [_P, _I32, ctypes.POINTER(_I32), _P]),
    "mcinv_check_convergence": (_I32, [_P, _I64, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "mcinv_get_info": (_I32, [_P, ctypes.POINTER(mcinv_info)]),
    "mcinv_reset_profile": (_I32, [_P]),
    "mcinv_noise_values": (_I32, [_I32, _U64, _U32, _I32, _I32, _I64, _P, _P, _P, _P]),
    "mcinv_last_error": (ctypes.c_char_p, [_P]),
    "mcinv_batch_create": (_I32, [ctypes.POINTER(mcinv_batch_config), _I64, ctypes.POINTER(_P)]),
    "mcinv_batch_destroy": (None, [_P]),
    "mcinv_batch_load_csr": (_I32, [_P, _I64, _I64, _I64, _P, _P, _P]),
    "mcinv_batch_set_requested": (_I32, [_P, _U32, _I32, _I64]),
    "mcinv_batch_set_block": (_I32, [_P, _I64, _P, _P]),
    "mcinv_batch_burn_in": (_I32, [_P, _I64]),
    "mcinv_batch_sample": (_I32, [_P, _I64]),
    "mcinv_batch_burn_in_coupled": (_I32, [_P, _D, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_D)]),
    "mcinv_batch_sample_until": (_I32, [_P, _D, _I64, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_D)]),
    "mcinv_batch_sample_until_each": (_I32, [_P, _D, _I64, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_D)]),
    "mcinv_batch_matrix_samples": (_I32, [_P, _P, _P]),
    "mcinv_batch_read_estimates": (_I32, [_P, _I64, _U32, _P, _P, _I64]),
    "mcinv_batch_read_state": (_I32, [_P, _I64, _I32, _P, _I64]),
    "mcinv_batch_read_labels": (_I32, [_P, _I64, _P, _P, _I64]),
    "mcinv_batch_autotune": (_I32, [_P, _I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                    ctypes.POINTER(_D)]),
    "mcinv_batch_get_info": (_I32, [_P, ctypes.POINTER(mcinv_batch_info)]),
    "mcinv_batch_last_error": (ctypes.c_char_p, [_P]),
    "mcinv_features_noalloc": (_I32, [_I32, _I64, _I64, _P, _P, _P, _P, _P]),
    "mcinv_features": (_I32, [_I32, _I64, _I64, _P, _P, _P, _P]),
    "mcinv_mlp_create": (_I32, [_I32, ctypes.POINTER(_P)]),
    "mcinv_mlp_destroy": (None, [_P]),
    "mcinv_mlp_set_params": (_I32, [_P, _P]),
    "mcinv_mlp_get_params": (_I32, [_P, _P]),
    "mcinv_mlp_set_normalization": (_I32, [_P, _P, _P]),
    "mcinv_mlp_set_data": (_I32, [_P, _P, _P, _P, _I64]),
    "mcinv_mlp_fit_normalization": (_I32, [_P, _P, _P]),
    "mcinv_mlp_label_weights": (_I32, [_I64, _P, _D, _P]),
    "mcinv_mlp_gradients": (_I32, [_P, _P, _I32, _P, ctypes.POINTER(ctypes.c_float)]),
    "mcinv_mlp_train": (_I32, [_P, _I64, _I32, ctypes.c_float, _U64, _P]),
    "mcinv_mlp_predict": (_I32, [_P, _P, _I64, _P]),
    "mcinv_mlp_last_error": (ctypes.c_char_p, [_P]),
    "mcinv_gate_fit": (_I32, [ctypes.POINTER(mcinv_gate_config), _I64, _P, _P, _P, _P, ctypes.POINTER(_P)]),
    "mcinv_gate_apply": (_I32, [_P, _I64, _P, _P]),
    "mcinv_mlp_estimate_matrix": (_I32, [_P, _P, _I64, _I64, _P, _P, _P, _P, _P]),
    "mcinv_gate_read": (_I32, [_P, _P, _P, _P, _P, _P, _P]),
    "mcinv_gate_destroy": (None, [_P]),
    "mcinv_gate_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load ``libmcinv.so``.  There is no fallback: a missing library is an error."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(ctx, status):
    if status != MCINV_OK:
        msg = lib().mcinv_last_error(ctx)
        raise McinvError(status, msg.decode() if msg else "")
    return status


def mcinv_last_error(ctx=None):
    m = lib().mcinv_last_error(ctx)
    return m.decode() if m else ""


def mcinv_create(device=0, sweep_dtype=MCINV_R32, moments=MCINV_MOMENTS_FP64, noise=MCINV_NOISE_NORMAL,
                 n_pairs=1, n_groups=1, stream_id=0, seed=0, stream=None, profile=False, pass_tiles=0,
                 hermitian=False, xcd_order=0, pair_offset=0, stores=0):
    cfg = mcinv_config(device, sweep_dtype, moments, noise, n_pairs, n_groups, stream_id,
                       seed & 0xFFFFFFFFFFFFFFFF, stream, 1 if profile else 0, int(pass_tiles), int(xcd_order),
                       1 if hermitian else 0, int(pair_offset), int(stores))
    h = ctypes.c_void_p()
    _check(None, lib().mcinv_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h


def mcinv_destroy(ctx):
    lib().mcinv_destroy(ctx)


def mcinv_load_csr(ctx, n, nnz, row_ptr, col_idx, values):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if np.iscomplexobj(values):
        v = np.ascontiguousarray(values, dtype=np.complex128)
        vd = MCINV_C128
    else:
        v = np.ascontiguousarray(values, dtype=np.float64)
        vd = MCINV_R64
    _check(ctx, lib().mcinv_load_csr(ctx, int(n), int(nnz), _ptr(rp), _ptr(ci), _ptr(v), vd))


def _idx(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int64)


def mcinv_set_requested(ctx, flags, block_rows=None, block_cols=None, entry_i=None, entry_j=None):
    br, bc, ei, ej = _idx(block_rows), _idx(block_cols), _idx(entry_i), _idx(entry_j)
    _check(ctx, lib().mcinv_set_requested(ctx, flags, _ptr(br), 0 if br is None else br.size, _ptr(bc),
                                          0 if bc is None else bc.size, _ptr(ei), _ptr(ej),
                                          0 if ei is None else ei.size))


def mcinv_burn_in(ctx, sweeps):
    _check(ctx, lib().mcinv_burn_in(ctx, int(sweeps)))


def mcinv_burn_in_coupled(ctx, tol=5e-5, max_sweeps=10000):
    n = ctypes.c_int64(0)
    dz = ctypes.c_double(0)
    dw = ctypes.c_double(0)
    _check(ctx, lib().mcinv_burn_in_coupled(ctx, float(tol), int(max_sweeps), ctypes.byref(n), ctypes.byref(dz),
                                            ctypes.byref(dw)))
    return n.value, dz.value, dw.value


def mcinv_sample(ctx, sweeps):
    _check(ctx, lib().mcinv_sample(ctx, int(sweeps)))


def mcinv_sample_until(ctx, rel_se, max_sweeps, check_every):
    done = ctypes.c_int64(0)
    ach = ctypes.c_double(0)
    _check(ctx, lib().mcinv_sample_until(ctx, float(rel_se), int(max_sweeps), int(check_every),
                                         ctypes.byref(done), ctypes.byref(ach)))
    return done.value, ach.value


def mcinv_sample_until_trace(ctx, rel_se, max_sweeps, check_every):
    done = ctypes.c_int64(0)
    ach = ctypes.c_double(0)
    _check(ctx, lib().mcinv_sample_until_trace(ctx, float(rel_se), int(max_sweeps), int(check_every),
                                               ctypes.byref(done), ctypes.byref(ach)))
    return done.value, ach.value


def mcinv_read_estimates(ctx, quantity, count, is_complex):
    est = np.empty(count * (2 if is_complex else 1), dtype=np.float64)
    se = np.empty(count, dtype=np.float64)
    _check(ctx, lib().mcinv_read_estimates(ctx, quantity, _ptr(est), _ptr(se), int(count)))
    if is_complex:
        est = est.view(np.complex128)
    return est, se


def mcinv_read_trace_stats(ctx, quantity):
    """Geyer statistics of the trace series: dict of mean, variance (gamma_0),
    sigma2, n_eff, se and samples."""
    st = np.empty(9, dtype=np.float64)
    _check(ctx, lib().mcinv_read_trace_stats(ctx, quantity, _ptr(st)))
    return {"mean": complex(st[0], st[1]), "var": float(st[2]), "sigma2": float(st[3]), "n_eff": float(st[4]),
            "se": float(st[5]), "samples": int(st[6]), "var_re": float(st[7]), "var_im": float(st[8])}


def mcinv_read_state(ctx, which, n, P, sweep_dtype):
    out = np.empty((n, P), dtype=NP_STATE[sweep_dtype])
    _check(ctx, lib().mcinv_read_state(ctx, which, _ptr(out), out.nbytes))
    return out


def mcinv_write_state(ctx, which, state, sweep_dtype):
    a = np.ascontiguousarray(state, dtype=NP_STATE[sweep_dtype])
    _check(ctx, lib().mcinv_write_state(ctx, which, _ptr(a), a.nbytes))


def mcinv_set_trace_matrix(ctx, n, row_ptr, col_idx, values):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if np.iscomplexobj(values):
        v = np.ascontiguousarray(values, dtype=np.complex128).view(np.float64)
        vd = MCINV_C128
    else:
        v = np.ascontiguousarray(values, dtype=np.float64)
        vd = MCINV_R64
    if rp.size != n + 1:
        raise ValueError("row_ptr must have n + 1 entries")
    _check(ctx, lib().mcinv_set_trace_matrix(ctx, int(rp[-1]), _ptr(rp), _ptr(ci), _ptr(v), vd))


def mcinv_save(ctx, path):
    _check(ctx, lib().mcinv_save(ctx, os.fsencode(path)))


def mcinv_restore(ctx, path):
    _check(ctx, lib().mcinv_restore(ctx, os.fsencode(path)))


def mcinv_set_stop_rows(ctx, rows=None):
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    _check(ctx, lib().mcinv_set_stop_rows(ctx, _ptr(r), 0 if r is None else int(r.size)))


def mcinv_get_permutation(ctx, n):
    perm = np.empty(n, dtype=np.int64)
    color = np.empty(n, dtype=np.int32)
    _check(ctx, lib().mcinv_get_permutation(ctx, _ptr(perm), _ptr(color)))
    return perm, color


def mcinv_tune_launch(ctx, sweeps_per_trial=2):
    o = ctypes.c_int32(0)
    ms = np.zeros(4, dtype=np.float64)
    _check(ctx, lib().mcinv_tune_launch(ctx, int(sweeps_per_trial), ctypes.byref(o), _ptr(ms)))
    return o.value, ms


def mcinv_check_convergence(ctx, iters):
    rt = ctypes.c_double(0)
    rs = ctypes.c_double(0)
    _check(ctx, lib().mcinv_check_convergence(ctx, int(iters), ctypes.byref(rt), ctypes.byref(rs)))
    return rt.value, rs.value


def mcinv_get_info(ctx):
    info = mcinv_info()
    _check(ctx, lib().mcinv_get_info(ctx, ctypes.byref(info)))
    return info.as_dict()


def mcinv_reset_profile(ctx):
    _check(ctx, lib().mcinv_reset_profile(ctx))


def mcinv_noise_values(device, seed, stream_id, noise, dtype, row, sweep, pair):
    r = np.ascontiguousarray(row, dtype=np.int64).ravel()
    k = np.ascontiguousarray(sweep, dtype=np.int64).ravel()
    p = np.ascontiguousarray(pair, dtype=np.int64).ravel()
    out = np.empty(r.size, dtype=np.float64)
    _check(None, lib().mcinv_noise_values(device, seed & 0xFFFFFFFFFFFFFFFF, stream_id, noise, dtype, r.size,
                                          _ptr(r), _ptr(k), _ptr(p), _ptr(out)))
    return out


# ---------------------------------------------------------------- batched --
def _bcheck(b, status):
    if status != MCINV_OK:
        msg = lib().mcinv_batch_last_error(b)
        raise McinvError(status, msg.decode() if msg else "")
    return status


def mcinv_batch_last_error(b=None):
    m = lib().mcinv_batch_last_error(b)
    return m.decode() if m else ""


MCINV_SCHEDULE_PHASED, MCINV_SCHEDULE_PERSISTENT = 0, 1


def mcinv_batch_create(n_matrices, device=0, noise=MCINV_NOISE_NORMAL, n_pairs=64, n_groups=16, rows_per_item=0,
                       grab=0, seed=0, stream=None, schedule=MCINV_SCHEDULE_PHASED):
    cfg = mcinv_batch_config(device, noise, n_pairs, n_groups, rows_per_item, grab, schedule,
                             seed & 0xFFFFFFFFFFFFFFFF, stream)
    h = ctypes.c_void_p()
    _bcheck(None, lib().mcinv_batch_create(ctypes.byref(cfg), int(n_matrices), ctypes.byref(h)))
    return h


def mcinv_batch_destroy(b):
    lib().mcinv_batch_destroy(b)


def mcinv_batch_load_csr(b, m, n, nnz, row_ptr, col_idx, values):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = np.ascontiguousarray(values, dtype=np.float64)
    _bcheck(b, lib().mcinv_batch_load_csr(b, int(m), int(n), int(nnz), _ptr(rp), _ptr(ci), _ptr(v)))


def mcinv_batch_set_requested(b, flags, block_dim=0, expected_samples=1):
    _bcheck(b, lib().mcinv_batch_set_requested(b, flags, int(block_dim), int(expected_samples)))


def mcinv_batch_set_block(b, m, rows, cols):
    r = np.ascontiguousarray(rows, dtype=np.int64)
    c = np.ascontiguousarray(cols, dtype=np.int64)
    _bcheck(b, lib().mcinv_batch_set_block(b, int(m), _ptr(r), _ptr(c)))


def mcinv_batch_burn_in(b, sweeps):
    _bcheck(b, lib().mcinv_batch_burn_in(b, int(sweeps)))


def mcinv_batch_burn_in_coupled(b, tol=5e-5, max_sweeps=10000):
    n = ctypes.c_int64(0)
    d = ctypes.c_double(0)
    _bcheck(b, lib().mcinv_batch_burn_in_coupled(b, float(tol), int(max_sweeps), ctypes.byref(n), ctypes.byref(d)))
    return n.value, d.value


def mcinv_batch_sample(b, sweeps):
    _bcheck(b, lib().mcinv_batch_sample(b, int(sweeps)))


def mcinv_batch_sample_until(b, rel_se, max_sweeps, check_every):
    done = ctypes.c_int64(0)
    ach = ctypes.c_double(0)
    _bcheck(b, lib().mcinv_batch_sample_until(b, float(rel_se), int(max_sweeps), int(check_every),
                                              ctypes.byref(done), ctypes.byref(ach)))
    return done.value, ach.value


def mcinv_batch_sample_until_each(b, rel_se, max_sweeps, check_every):
    done = ctypes.c_int64(0)
    ach = ctypes.c_double(0)
    _bcheck(b, lib().mcinv_batch_sample_until_each(b, float(rel_se), int(max_sweeps), int(check_every),
                                                   ctypes.byref(done), ctypes.byref(ach)))
    return done.value, ach.value


def mcinv_batch_matrix_samples(b, n_matrices):
    samples = np.zeros(n_matrices, dtype=np.int64)
    active = np.zeros(n_matrices, dtype=np.uint8)
    _bcheck(b, lib().mcinv_batch_matrix_samples(b, _ptr(samples), _ptr(active)))
    return samples, active.astype(bool)


def mcinv_batch_read_estimates(b, m, quantity, count):
    est = np.empty(count, dtype=np.float64)
    se = np.empty(count, dtype=np.float64)
    _bcheck(b, lib().mcinv_batch_read_estimates(b, int(m), quantity, _ptr(est), _ptr(se), int(count)))
    return est, se


def mcinv_batch_read_labels(b, m, count):
    y = np.empty(count, dtype=np.float64)
    y_se = np.empty(count, dtype=np.float64)
    _bcheck(b, lib().mcinv_batch_read_labels(b, int(m), _ptr(y), _ptr(y_se), int(count)))
    return y, y_se


def mcinv_batch_read_state(b, m, which, n, P):
    out = np.empty((n, P), dtype=np.float32)
    _bcheck(b, lib().mcinv_batch_read_state(b, int(m), which, _ptr(out), out.nbytes))
    return out


def mcinv_batch_autotune(b, sweeps_per_trial=2):
    sc = ctypes.c_int32(0)
    r = ctypes.c_int32(0)
    g = ctypes.c_int32(0)
    ms = ctypes.c_double(0)
    _bcheck(b, lib().mcinv_batch_autotune(b, int(sweeps_per_trial), ctypes.byref(sc), ctypes.byref(r),
                                          ctypes.byref(g), ctypes.byref(ms)))
    return sc.value, r.value, g.value, ms.value


def mcinv_batch_get_info(b):
    info = mcinv_batch_info()
    _bcheck(b, lib().mcinv_batch_get_info(b, ctypes.byref(info)))
    return info.as_dict()


# -------------------------------------------------------------- surrogate --
MCINV_N_FEATURES = 32
MCINV_MLP_PARAMS = 20865


def mcinv_features(device, n, nnz, row_ptr, col_idx, values):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = np.ascontiguousarray(values, dtype=np.float64)
    out = np.empty((int(n), MCINV_N_FEATURES), dtype=np.float32)
    _check(None, lib().mcinv_features(int(device), int(n), int(nnz), _ptr(rp), _ptr(ci), _ptr(v), _ptr(out)))
    return out


def mcinv_features_noalloc(device, n, nnz, row_ptr, col_idx, values, out, stream=None):
    """Device-array form (``mcinv_features_noalloc``): row_ptr, col_idx, values
    and out are device addresses (ints, e.g. torch ``data_ptr()``)."""
    _check(None, lib().mcinv_features_noalloc(int(device), int(n), int(nnz), ctypes.c_void_p(row_ptr),
                                              ctypes.c_void_p(col_idx), ctypes.c_void_p(values),
                                              ctypes.c_void_p(out), stream))


def _mcheck(m, status):
    if status != MCINV_OK:
        msg = lib().mcinv_mlp_last_error(m)
        raise McinvError(status, msg.decode() if msg else "")
    return status


def mcinv_mlp_last_error(m=None):
    s = lib().mcinv_mlp_last_error(m)
    return s.decode() if s else ""


def mcinv_mlp_create(device=0):
    h = ctypes.c_void_p()
    _mcheck(None, lib().mcinv_mlp_create(int(device), ctypes.byref(h)))
    return h


def mcinv_mlp_destroy(m):
    lib().mcinv_mlp_destroy(m)


def _f32(a, size=None):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if size is not None and a.size != size:
        raise ValueError(f"expected {size} values, got {a.size}")
    return a


def mcinv_mlp_set_params(m, params):
    p = _f32(params, MCINV_MLP_PARAMS)
    _mcheck(m, lib().mcinv_mlp_set_params(m, _ptr(p)))


def mcinv_mlp_get_params(m):
    out = np.empty(MCINV_MLP_PARAMS, dtype=np.float32)
    _mcheck(m, lib().mcinv_mlp_get_params(m, _ptr(out)))
    return out


def mcinv_mlp_set_normalization(m, mean, inv_std):
    a = _f32(mean, MCINV_N_FEATURES)
    b = _f32(inv_std, MCINV_N_FEATURES)
    _mcheck(m, lib().mcinv_mlp_set_normalization(m, _ptr(a), _ptr(b)))


def mcinv_mlp_set_data(m, X, y, w):
    X = _f32(X)
    y = _f32(y)
    w = _f32(w)
    N = y.size
    if X.size != N * MCINV_N_FEATURES or w.size != N:
        raise ValueError("X must be [N][32], y and w [N]")
    _mcheck(m, lib().mcinv_mlp_set_data(m, _ptr(X), _ptr(y), _ptr(w), int(N)))


def mcinv_mlp_fit_normalization(m):
    mean = np.empty(MCINV_N_FEATURES, dtype=np.float32)
    inv = np.empty(MCINV_N_FEATURES, dtype=np.float32)
    _mcheck(m, lib().mcinv_mlp_fit_normalization(m, _ptr(mean), _ptr(inv)))
    return mean, inv


def mcinv_mlp_label_weights(y_se, eps=1e-6):
    se = np.ascontiguousarray(y_se, dtype=np.float64)
    w = np.empty(se.size, dtype=np.float32)
    _mcheck(None, lib().mcinv_mlp_label_weights(int(se.size), _ptr(se), float(eps), _ptr(w)))
    return w


def mcinv_mlp_gradients(m, rows):
    r = np.ascontiguousarray(rows, dtype=np.int64)
    g = np.empty(MCINV_MLP_PARAMS, dtype=np.float32)
    loss = ctypes.c_float(0)
    _mcheck(m, lib().mcinv_mlp_gradients(m, _ptr(r), int(r.size), _ptr(g), ctypes.byref(loss)))
    return g, loss.value


def mcinv_mlp_train(m, steps, batch_rows, lr, seed):
    hist = np.empty(max(int(steps), 1), dtype=np.float32)
    _mcheck(m, lib().mcinv_mlp_train(m, int(steps), int(batch_rows), float(lr), seed & 0xFFFFFFFFFFFFFFFF,
                                      _ptr(hist)))
    return hist[:int(steps)]


def mcinv_mlp_predict(m, X):
    X = _f32(X)
    N = X.size // MCINV_N_FEATURES
    out = np.empty(N, dtype=np.float32)
    _mcheck(m, lib().mcinv_mlp_predict(m, _ptr(X), int(N), _ptr(out)))
    return out


def _gcheck(status):
    if status != MCINV_OK:
        msg = lib().mcinv_gate_last_error()
        raise McinvError(status, msg.decode() if msg else "")
    return status


def mcinv_gate_fit(X, pred, y, y_se, feature_a, feature_b, bins, min_rows, tol, ucb_z=0.0):
    X = _f32(X)
    N = X.size // MCINV_N_FEATURES
    pr = np.ascontiguousarray(pred, dtype=np.float64)
    yy = np.ascontiguousarray(y, dtype=np.float64)
    se = np.ascontiguousarray(y_se, dtype=np.float64)
    if pr.size != N or yy.size != N or se.size != N:
        raise ValueError("pred, y and y_se need one value per row of X")
    cfg = mcinv_gate_config(int(feature_a), int(feature_b), int(bins), int(min_rows), float(tol), float(ucb_z))
    h = ctypes.c_void_p()
    _gcheck(lib().mcinv_gate_fit(ctypes.byref(cfg), int(N), _ptr(X), _ptr(pr), _ptr(yy), _ptr(se),
                                 ctypes.byref(h)))
    return h


def mcinv_gate_apply(g, X):
    X = _f32(X)
    N = X.size // MCINV_N_FEATURES
    out = np.empty(N, dtype=np.uint8)
    _gcheck(lib().mcinv_gate_apply(g, int(N), _ptr(X), _ptr(out)))
    return out


def mcinv_mlp_estimate_matrix(m, g, n, nnz, row_ptr, col_idx, values):
    """(estimates of (C^-1)_ii float64[n], gate fallback uint8[n]) for a real
    CSR matrix, its features computed and consumed on the device."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    v = np.ascontiguousarray(values, dtype=np.float64)
    est = np.empty(int(n), dtype=np.float64)
    fb = np.empty(int(n), dtype=np.uint8)
    _mcheck(m, lib().mcinv_mlp_estimate_matrix(m, g, int(n), int(nnz), _ptr(rp), _ptr(ci), _ptr(v), _ptr(est),
                                               _ptr(fb)))
    return est, fb


def mcinv_gate_read(g, bins):
    ea = np.empty(max(bins - 1, 0), dtype=np.float64)
    eb = np.empty(max(bins - 1, 0), dtype=np.float64)
    err = np.empty(bins * bins, dtype=np.float64)
    cnt = np.empty(bins * bins, dtype=np.int64)
    fb = np.empty(bins * bins, dtype=np.uint8)
    rng = np.empty(4, dtype=np.float64)
    _gcheck(lib().mcinv_gate_read(g, _ptr(ea), _ptr(eb), _ptr(err), _ptr(cnt), _ptr(fb), _ptr(rng)))
    return {"edges_a": ea, "edges_b": eb, "err": err, "count": cnt, "fallback": fb.astype(bool),
            "range_a": (float(rng[0]), float(rng[1])), "range_b": (float(rng[2]), float(rng[3]))}


def mcinv_gate_destroy(g):
    lib().mcinv_gate_destroy(g)


def mcinv_gate_last_error():
    m = lib().mcinv_gate_last_error()
    return m.decode() if m else ""

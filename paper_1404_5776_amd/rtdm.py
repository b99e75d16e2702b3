"""Python binding of librtdm.so (include/rtdm.h): the C names, argument marshalling only.

Every step of the propagation runs in the library's HIP kernels; this module
only converts numpy arrays / torch tensors to pointers and status codes to
exceptions.  It fails loudly (RuntimeError at load) when the library has not
been built: there is no fallback path.
"""

from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtdm.so")

MAT = {"S": 0, "H0": 1, "H": 2, "X": 3, "A": 4, "U": 5, "K": 6, "W": 7}
PROD = {"XH": 0, "AT": 1, "UK": 2, "WU": 3, "SX": 4, "UV": 5, "ZX": 6}
HMODEL = {"fixed": 0, "mulliken": 1}
INV_START = {"block_jacobi": 0, "cold": 1, "previous": 2, "learned": 3}
PRECISION = {"fp64": 0, "fp32": 1, "fp32_taylor": 2, "bf16x3": 3, "fp16x2": 4, "bf16x3_taylor": 5,
             "fp16x2_taylor": 6}
PROPAGATOR = {"em": 0, "etrs": 1, "m4": 2}

STATUS = {0: "RTDM_OK", -1: "RTDM_E_ARG", -2: "RTDM_E_STATE", -3: "RTDM_E_OOM", -4: "RTDM_E_HIP",
          -5: "RTDM_E_NOCONV", -6: "RTDM_E_NUMERIC", -7: "RTDM_E_UNSUPPORTED"}

EXPORTED = ["rtdm_default_options", "rtdm_create", "rtdm_destroy", "rtdm_set_geometry",
            "rtdm_set_ranges", "rtdm_pattern", "rtdm_upload", "rtdm_upload_coo", "rtdm_download",
            "rtdm_apply_kick", "rtdm_build_inverse", "rtdm_step", "rtdm_observables",
            "rtdm_dipole_trace", "rtdm_unitarity", "rtdm_inverse_error", "rtdm_multiply", "rtdm_multiply_noalloc",
            "rtdm_schedule_stats",
            "rtdm_timing", "rtdm_timing_stats", "rtdm_inverse_info", "rtdm_mlp_params", "rtdm_mlp_init",
            "rtdm_mlp_set_weights", "rtdm_mlp_get_weights", "rtdm_mlp_collect", "rtdm_mlp_clear",
            "rtdm_mlp_train", "rtdm_mlp_loss_grad", "rtdm_mlp_step", "rtdm_mlp_predict", "rtdm_set_groups",
            "rtdm_apply_kick_groups", "rtdm_group_trace", "rtdm_apply_kicks", "rtdm_select_kick", "rtdm_unbind_workspace", "rtdm_reserve_trace", "rtdm_set_allocator",
            "rtdm_batch_create", "rtdm_batch_step", "rtdm_batch_last_error", "rtdm_batch_destroy", "rtdm_autotune", "rtdm_set_field",
            "rtdm_spectrum", "rtdm_workspace_size", "rtdm_bind_workspace", "rtdm_ground_state",
            "rtdm_get_state", "rtdm_set_state", "rtdm_last_error"]


class RtdmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("taylor_order", ctypes.c_int), ("unit_check_every", ctypes.c_int),
                ("precision", ctypes.c_int), ("h_model", ctypes.c_int), ("h_gain", ctypes.c_double),
                ("inv_start", ctypes.c_int), ("inv_tol", ctypes.c_double),
                ("inv_max_iter", ctypes.c_int), ("taylor_low_from", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("propagator", ctypes.c_int), ("sc_steps", ctypes.c_int), ("sc_iters", ctypes.c_int),
                ("unit_tol", ctypes.c_double), ("graph_steps", ctypes.c_int), ("n_kicks", ctypes.c_int),
                ("xh_every_step", ctypes.c_int)]


_lib = None


def load():
    """Load librtdm.so (RuntimeError if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
    # PyTorch first: it ships its own HIP runtime under the same soname, and the
    # process must hold one runtime (the first loaded serves both), so that
    # torch's device memory and streams are the library's too
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    sig = {
        "rtdm_default_options": [P],
        "rtdm_create": [ctypes.POINTER(P), I, P],
        "rtdm_destroy": [P],
        "rtdm_set_geometry": [P, I64, P, P],
        "rtdm_set_ranges": [P, D, D, D],
        "rtdm_pattern": [P, I, P, P, P, P],
        "rtdm_upload": [P, I, P, I, I, P],
        "rtdm_upload_coo": [P, I, I64, P, P, P, I, P],
        "rtdm_download": [P, I, P, I, P],
        "rtdm_apply_kick": [P, P, P],
        "rtdm_build_inverse": [P, P, P, P],
        "rtdm_step": [P, D, I64, P],
        "rtdm_observables": [P, P, P],
        "rtdm_dipole_trace": [P, P, I64, P],
        "rtdm_unitarity": [P, P, P],
        "rtdm_inverse_error": [P, P, P],
        "rtdm_multiply": [P, I, I, I, I, I, D, D, P],
        "rtdm_multiply_noalloc": [P, I, I, I, I, I, D, D, P],
        "rtdm_schedule_stats": [P, I, P, P],
        "rtdm_timing": [P, I],
        "rtdm_timing_stats": [P, I, P, P, P],
        "rtdm_inverse_info": [P, P, P],
        "rtdm_mlp_params": [P, P, P, P, P],
        "rtdm_mlp_init": [P, ctypes.c_uint64],
        "rtdm_mlp_set_weights": [P, P, I64],
        "rtdm_mlp_get_weights": [P, P, I64],
        "rtdm_mlp_collect": [P, I64, ctypes.c_uint64, P],
        "rtdm_mlp_clear": [P],
        "rtdm_mlp_train": [P, I, I, D, ctypes.c_uint64, P],
        "rtdm_mlp_loss_grad": [P, I64, P, P, P, P],
        "rtdm_mlp_step": [P, I64, P, P, D, P],
        "rtdm_mlp_predict": [P, I64, P, P],
        "rtdm_set_groups": [P, I64, P],
        "rtdm_apply_kick_groups": [P, P, P],
        "rtdm_group_trace": [P, P, I64, P],
        "rtdm_apply_kicks": [P, P, P],
        "rtdm_unbind_workspace": [P],
        "rtdm_set_allocator": [P, P, P, P],
        "rtdm_reserve_trace": [P, I64],
        "rtdm_batch_create": [P, P, I, I],
        "rtdm_batch_step": [P, D, I64, P],
        "rtdm_batch_last_error": [P],
        "rtdm_batch_destroy": [P],
        "rtdm_select_kick": [P, I],
        "rtdm_autotune": [P, P, P, P],
        "rtdm_set_field": [P, P, D, D],
        "rtdm_spectrum": [P, I64, P, P, D, I64, P, P, P, P],
        "rtdm_workspace_size": [P, P],
        "rtdm_bind_workspace": [P, P, ctypes.c_size_t],
        "rtdm_ground_state": [P, D, D, ctypes.c_int, P, P, P, P],
        "rtdm_get_state": [P, P, I64, P],
        "rtdm_set_state": [P, P, I64, P],
        "rtdm_last_error": [P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name in ("rtdm_last_error", "rtdm_batch_last_error") else ctypes.c_int
    _lib = L
    return L


def _check(ctx, rc: int):
    if rc != 0:
        msg = load().rtdm_last_error(ctx)
        raise RtdmError(rc, msg.decode() if msg else "")


def _stream(stream) -> Optional[int]:
    if stream is None:
        torch = sys.modules.get("torch")
        if torch is not None and torch.cuda.is_initialized():
            return torch.cuda.current_stream().cuda_stream
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _mat(m) -> int:
    return MAT[m] if isinstance(m, str) else int(m)


def _prod(p) -> int:
    return PROD[p] if isinstance(p, str) else int(p)


# ------------------------------------------------------------------ C names

def rtdm_default_options() -> Options:
    o = Options()
    load().rtdm_default_options(ctypes.byref(o))
    return o


def rtdm_create(device: int = 0, options: Optional[Options] = None):
    L = load()
    h = ctypes.c_void_p()
    rc = L.rtdm_create(ctypes.byref(h), int(device), ctypes.byref(options) if options is not None else None)
    if rc != 0:
        raise RtdmError(rc, "rtdm_create failed")
    return h


def rtdm_destroy(ctx) -> None:
    _check(ctx, load().rtdm_destroy(ctx))


def rtdm_set_geometry(ctx, xyz: np.ndarray, nbf: np.ndarray) -> None:
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    nbf = np.ascontiguousarray(nbf, dtype=np.int32)
    _check(ctx, load().rtdm_set_geometry(ctx, xyz.shape[0], _p(xyz), _p(nbf)))


def rtdm_set_ranges(ctx, R_HS: float, R_P: float, R_K: float) -> None:
    _check(ctx, load().rtdm_set_ranges(ctx, float(R_HS), float(R_P), float(R_K)))


def rtdm_pattern(ctx, mat) -> Tuple[np.ndarray, np.ndarray]:
    n = ctypes.c_int64()
    nnz = ctypes.c_int64()
    rp = ctypes.POINTER(ctypes.c_int64)()
    ci = ctypes.POINTER(ctypes.c_int32)()
    _check(ctx, load().rtdm_pattern(ctx, _mat(mat), ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(rp),
                                    ctypes.byref(ci)))
    row_ptr = np.ctypeslib.as_array(rp, shape=(n.value + 1,)).copy()
    col = np.ctypeslib.as_array(ci, shape=(nnz.value,)).copy() if nnz.value else np.zeros(0, np.int32)
    return row_ptr, col


def rtdm_upload(ctx, mat, data, stream=None) -> None:
    """data: numpy (host) or torch CUDA tensor, real float64 or complex128, blocks in pattern order."""
    if hasattr(data, "data_ptr"):
        is_c = int(data.is_complex())
        if not data.is_contiguous():
            raise ValueError("tensor must be contiguous")
        _check(ctx, load().rtdm_upload(ctx, _mat(mat), ctypes.c_void_p(data.data_ptr()), is_c,
                                       int(data.is_cuda), _stream(stream)))
        return
    is_c = int(np.iscomplexobj(data))
    arr = np.ascontiguousarray(data, dtype=np.complex128 if is_c else np.float64)
    _check(ctx, load().rtdm_upload(ctx, _mat(mat), _p(arr), is_c, 0, _stream(stream)))


def rtdm_upload_coo(ctx, mat, rows, cols, data, stream=None) -> None:
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    is_c = int(np.iscomplexobj(data))
    arr = np.ascontiguousarray(data, dtype=np.complex128 if is_c else np.float64)
    _check(ctx, load().rtdm_upload_coo(ctx, _mat(mat), rows.size, _p(rows), _p(cols), _p(arr), is_c,
                                       _stream(stream)))


def rtdm_download(ctx, mat, b: int, out=None, stream=None):
    """Blocks of a slot as complex128 (nnzb, b, b); into `out` (torch CUDA tensor) if given."""
    if out is not None:
        _check(ctx, load().rtdm_download(ctx, _mat(mat), ctypes.c_void_p(out.data_ptr()), 1, _stream(stream)))
        return out
    _, col = rtdm_pattern(ctx, mat)
    arr = np.empty((col.size, b, b), dtype=np.complex128)
    _check(ctx, load().rtdm_download(ctx, _mat(mat), _p(arr), 0, _stream(stream)))
    return arr


def rtdm_download_mixed(ctx, mat, nbf, stream=None):
    """Blocks of a slot with per-atom sizes nbf: (flat complex128 data, block
    offsets); block p (rtdm_pattern order) is data[off[p]:off[p+1]], row-major
    nbf_i x nbf_j."""
    rp, col = rtdm_pattern(ctx, mat)
    nbf = np.asarray(nbf, dtype=np.int64)
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    sizes = nbf[rows] * nbf[col]
    arr = np.empty(int(sizes.sum()), dtype=np.complex128)
    _check(ctx, load().rtdm_download(ctx, _mat(mat), _p(arr), 0, _stream(stream)))
    return arr, np.concatenate([[0], np.cumsum(sizes)])


def rtdm_apply_kick(ctx, kappa: Sequence[float], stream=None) -> None:
    k = np.ascontiguousarray(kappa, dtype=np.float64)
    _check(ctx, load().rtdm_apply_kick(ctx, _p(k), _stream(stream)))


def rtdm_build_inverse(ctx, stream=None) -> Tuple[int, float]:
    it = ctypes.c_int()
    r = ctypes.c_double()
    _check(ctx, load().rtdm_build_inverse(ctx, _stream(stream), ctypes.byref(it), ctypes.byref(r)))
    return it.value, r.value


def rtdm_step(ctx, dt: float, n_steps: int, stream=None) -> None:
    _check(ctx, load().rtdm_step(ctx, float(dt), int(n_steps), _stream(stream)))


def rtdm_observables(ctx, stream=None) -> np.ndarray:
    out = np.zeros(6)
    _check(ctx, load().rtdm_observables(ctx, _p(out), _stream(stream)))
    return out


def rtdm_dipole_trace(ctx, max_rows: int = 1 << 20) -> np.ndarray:
    rows = ctypes.c_int64()
    _check(ctx, load().rtdm_dipole_trace(ctx, None, 0, ctypes.byref(rows)))
    n = min(rows.value, max_rows)
    out = np.zeros((n, 7))
    _check(ctx, load().rtdm_dipole_trace(ctx, _p(out), n, ctypes.byref(rows)))
    return out


def rtdm_unitarity(ctx, stream=None) -> np.ndarray:
    out = np.zeros(3)
    _check(ctx, load().rtdm_unitarity(ctx, _p(out), _stream(stream)))
    return out


def rtdm_inverse_error(ctx, stream=None) -> np.ndarray:
    out = np.zeros(3)
    _check(ctx, load().rtdm_inverse_error(ctx, _p(out), _stream(stream)))
    return out


def rtdm_multiply(ctx, C, A, B, op_a: int = 0, op_b: int = 0, alpha: complex = 1.0, stream=None) -> None:
    a = complex(alpha)
    _check(ctx, load().rtdm_multiply(ctx, _mat(C), _mat(A), _mat(B), int(op_a), int(op_b), a.real, a.imag,
                                     _stream(stream)))


def rtdm_multiply_noalloc(ctx, C, A, B, op_a: int = 0, op_b: int = 0, alpha: complex = 1.0, stream=None) -> None:
    alpha = complex(alpha)
    _check(ctx, load().rtdm_multiply_noalloc(ctx, _mat(C), _mat(A), _mat(B), op_a, op_b, alpha.real, alpha.imag,
                                             _stream(stream)))


def rtdm_schedule_stats(ctx, prod) -> Tuple[int, int]:
    o = ctypes.c_int64()
    t = ctypes.c_int64()
    _check(ctx, load().rtdm_schedule_stats(ctx, _prod(prod), ctypes.byref(o), ctypes.byref(t)))
    return o.value, t.value


def rtdm_timing(ctx, enable: bool) -> None:
    _check(ctx, load().rtdm_timing(ctx, int(bool(enable))))


def rtdm_timing_stats(ctx, prod) -> Tuple[int, float, float]:
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    fl = ctypes.c_double()
    _check(ctx, load().rtdm_timing_stats(ctx, _prod(prod), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(fl)))
    return n.value, ms.value, fl.value


def rtdm_inverse_info(ctx) -> Tuple[int, int]:
    it = ctypes.c_int()
    fb = ctypes.c_int()
    _check(ctx, load().rtdm_inverse_info(ctx, ctypes.byref(it), ctypes.byref(fb)))
    return it.value, fb.value


def rtdm_mlp_params(ctx) -> Tuple[int, int, int, int]:
    n = ctypes.c_int64()
    i, h, o = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(ctx, load().rtdm_mlp_params(ctx, ctypes.byref(n), ctypes.byref(i), ctypes.byref(h), ctypes.byref(o)))
    return n.value, i.value, h.value, o.value


def rtdm_mlp_init(ctx, seed: int) -> None:
    _check(ctx, load().rtdm_mlp_init(ctx, int(seed)))


def rtdm_mlp_set_weights(ctx, w) -> None:
    a = np.ascontiguousarray(w, dtype=np.float32)
    _check(ctx, load().rtdm_mlp_set_weights(ctx, _p(a), a.size))


def rtdm_mlp_get_weights(ctx) -> np.ndarray:
    n = rtdm_mlp_params(ctx)[0]
    a = np.zeros(n, dtype=np.float32)
    _check(ctx, load().rtdm_mlp_get_weights(ctx, _p(a), n))
    return a


def rtdm_mlp_collect(ctx, max_samples: int, seed: int) -> int:
    t = ctypes.c_int64()
    _check(ctx, load().rtdm_mlp_collect(ctx, int(max_samples), int(seed), ctypes.byref(t)))
    return t.value


def rtdm_mlp_clear(ctx) -> None:
    _check(ctx, load().rtdm_mlp_clear(ctx))


def rtdm_mlp_train(ctx, epochs: int, batch: int, lr: float, seed: int) -> float:
    l = ctypes.c_double()
    _check(ctx, load().rtdm_mlp_train(ctx, int(epochs), int(batch), float(lr), int(seed), ctypes.byref(l)))
    return l.value


def rtdm_mlp_loss_grad(ctx, desc, target) -> Tuple[float, np.ndarray]:
    d = np.ascontiguousarray(desc, dtype=np.float32)
    t = np.ascontiguousarray(target, dtype=np.float32)
    g = np.zeros(rtdm_mlp_params(ctx)[0], dtype=np.float32)
    l = ctypes.c_double()
    _check(ctx, load().rtdm_mlp_loss_grad(ctx, d.shape[0], _p(d), _p(t), ctypes.byref(l), _p(g)))
    return l.value, g


def rtdm_mlp_step(ctx, desc, target, lr: float) -> float:
    d = np.ascontiguousarray(desc, dtype=np.float32)
    t = np.ascontiguousarray(target, dtype=np.float32)
    l = ctypes.c_double()
    _check(ctx, load().rtdm_mlp_step(ctx, d.shape[0], _p(d), _p(t), lr, ctypes.byref(l)))
    return l.value


def rtdm_mlp_predict(ctx, desc) -> np.ndarray:
    d = np.ascontiguousarray(desc, dtype=np.float32)
    out = rtdm_mlp_params(ctx)[3]
    y = np.zeros((d.shape[0], out), dtype=np.float32)
    _check(ctx, load().rtdm_mlp_predict(ctx, d.shape[0], _p(d), _p(y)))
    return y


def rtdm_set_groups(ctx, group_ptr) -> None:
    g = np.ascontiguousarray(group_ptr, dtype=np.int64)
    _check(ctx, load().rtdm_set_groups(ctx, g.size - 1, _p(g)))


def rtdm_apply_kick_groups(ctx, kappa, stream=None) -> None:
    k = np.ascontiguousarray(kappa, dtype=np.float64).reshape(-1)
    _check(ctx, load().rtdm_apply_kick_groups(ctx, _p(k), _stream(stream)))


def rtdm_apply_kicks(ctx, kappas, stream=None) -> None:
    k = np.ascontiguousarray(kappas, dtype=np.float64).reshape(-1)
    _check(ctx, load().rtdm_apply_kicks(ctx, _p(k), _stream(stream)))


def rtdm_batch_create(ctxs, graph_steps: int = 16):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value if isinstance(c, ctypes.c_void_p) else c for c in ctxs])
    h = ctypes.c_void_p()
    rc = load().rtdm_batch_create(ctypes.byref(h), arr, len(ctxs), int(graph_steps))
    if rc != 0:
        raise RtdmError(rc, "rtdm_batch_create failed")
    return h


def rtdm_batch_step(batch, dt: float, n_steps: int, stream=None) -> None:
    rc = load().rtdm_batch_step(batch, float(dt), int(n_steps), _stream(stream))
    if rc != 0:
        m = load().rtdm_batch_last_error(batch)
        raise RtdmError(rc, m.decode() if m else "")


def rtdm_batch_destroy(batch) -> None:
    load().rtdm_batch_destroy(batch)


def rtdm_unbind_workspace(ctx) -> None:
    _check(ctx, load().rtdm_unbind_workspace(ctx))


def rtdm_reserve_trace(ctx, rows: int) -> None:
    _check(ctx, load().rtdm_reserve_trace(ctx, int(rows)))


def rtdm_select_kick(ctx, k: int) -> None:
    _check(ctx, load().rtdm_select_kick(ctx, int(k)))


def rtdm_group_trace(ctx, n_groups: int, max_rows: int = 1 << 20) -> np.ndarray:
    rows = ctypes.c_int64()
    _check(ctx, load().rtdm_group_trace(ctx, None, 0, ctypes.byref(rows)))
    n = min(rows.value, max_rows)
    out = np.zeros((n, n_groups, 4))
    _check(ctx, load().rtdm_group_trace(ctx, _p(out), n, ctypes.byref(rows)))
    return out


def rtdm_autotune(ctx, stream=None) -> Tuple[int, int]:
    w = ctypes.c_int()
    t = ctypes.c_int()
    _check(ctx, load().rtdm_autotune(ctx, _stream(stream), ctypes.byref(w), ctypes.byref(t)))
    return w.value, t.value


def rtdm_set_field(ctx, E0, t0: float, sigma: float) -> None:
    e = np.ascontiguousarray(E0, dtype=np.float64)
    _check(ctx, load().rtdm_set_field(ctx, _p(e), float(t0), float(sigma)))


def rtdm_spectrum(ctx, P0, omega, gamma: float, kappa=None, group: int = -1, stream=None):
    """(alpha (n_w, 3) complex, strength (n_w,)) of the trace since the last kick."""
    p0 = np.ascontiguousarray(P0, dtype=np.float64)
    om = np.ascontiguousarray(omega, dtype=np.float64)
    al = np.zeros((om.size, 3, 2))
    sw = np.zeros(om.size)
    kp = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
    _check(ctx, load().rtdm_spectrum(ctx, int(group), _p(p0), None if kp is None else _p(kp), float(gamma),
                                     om.size, _p(om), _p(al), _p(sw), _stream(stream)))
    return al[..., 0] + 1j * al[..., 1], sw


def rtdm_workspace_size(ctx) -> int:
    n = ctypes.c_size_t()
    _check(ctx, load().rtdm_workspace_size(ctx, ctypes.byref(n)))
    return n.value


def rtdm_bind_workspace(ctx, ptr: int, nbytes: int) -> None:
    _check(ctx, load().rtdm_bind_workspace(ctx, ctypes.c_void_p(ptr), nbytes))


def rtdm_ground_state(ctx, n_occ: float, tol: float = 1e-10, max_iter: int = 64, stream=None):
    """(iterations, last idempotency measure, branch mask); K <- the ground state of H0."""
    it = ctypes.c_int()
    idem = ctypes.c_double()
    br = ctypes.c_uint64()
    _check(ctx, load().rtdm_ground_state(ctx, float(n_occ), float(tol), int(max_iter), _stream(stream),
                                         ctypes.byref(it), ctypes.byref(idem), ctypes.byref(br)))
    return it.value, idem.value, br.value


def rtdm_get_state(ctx, n_atoms: int, stream=None) -> np.ndarray:
    out = np.zeros(2 + 3 * n_atoms)
    _check(ctx, load().rtdm_get_state(ctx, _p(out), out.size, _stream(stream)))
    return out


def rtdm_set_state(ctx, state, stream=None) -> None:
    st = np.ascontiguousarray(state, dtype=np.float64)
    _check(ctx, load().rtdm_set_state(ctx, _p(st), st.size, _stream(stream)))


def rtdm_last_error(ctx) -> str:
    m = load().rtdm_last_error(ctx)
    return m.decode() if m else ""


# ------------------------------------------------------------------ convenience

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class TorchAllocator:
    """rtdm_set_allocator functions that take a context's device memory from
    PyTorch's caching allocator on one device (kept alive by the Context)."""

    def __init__(self, device: int):
        import torch
        torch.cuda.init()          # the caching allocator needs torch's runtime up
        _close_at_exit()
        self._torch = torch
        self.device = device
        self.last_error = None
        self.alloc_fn = _ALLOC_FN(self._alloc)
        self.free_fn = _FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            return self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device)
        except Exception as e:     # out of memory: the library reports RTDM_E_OOM
            self.last_error = repr(e)
            return None

    def _free(self, ptr, user):
        try:
            self._torch.cuda.caching_allocator_delete(ptr)
        except Exception:
            pass


def rtdm_set_allocator(ctx, allocator: TorchAllocator) -> None:
    rc = load().rtdm_set_allocator(ctx, allocator.alloc_fn, allocator.free_fn, None)
    if rc != 0 and allocator.last_error:
        raise RtdmError(rc, f"{rtdm_last_error(ctx)} ({allocator.last_error})")
    _check(ctx, rc)


_live_contexts = weakref.WeakSet()
_exit_hook = False


def _close_live_contexts():
    # give device memory back while PyTorch is still whole
    for c in list(_live_contexts):
        try:
            c.close()
        except Exception:
            pass


def _close_at_exit():
    """Register the closing of live contexts once, after torch is imported:
    exit handlers run last-registered first, so this one runs before
    PyTorch's own."""
    global _exit_hook
    if not _exit_hook:
        atexit.register(_close_live_contexts)
        _exit_hook = True


class Context:
    """Owns one rtdm context; `load_system` runs the set-up calls for a generated system."""

    def __init__(self, device: int = 0, memory: str = "torch", **opts):
        """memory: "torch" (default) takes every device buffer of the context
        from PyTorch's caching allocator (rtdm_set_allocator); "library" leaves
        it to the library's own hipMalloc.  Either way bind_workspace can move
        the buffers into one region; a later load moves them out first."""
        o = rtdm_default_options()
        for k, v in opts.items():
            if k == "h_model" and isinstance(v, str):
                v = HMODEL[v]
            if k == "inv_start" and isinstance(v, str):
                v = INV_START[v]
            if k == "precision" and isinstance(v, str):
                v = PRECISION[v]
            if k == "propagator" and isinstance(v, str):
                v = PROPAGATOR[v]
            setattr(o, k, v)
        if memory not in ("torch", "library"):
            raise ValueError(memory)
        self.options = o
        self.device = device
        self.workspace = None
        self.allocator = None
        self.h = rtdm_create(device, o)
        self.b = 0
        _live_contexts.add(self)
        if memory == "torch":
            self.allocator = TorchAllocator(device)
            rtdm_set_allocator(self.h, self.allocator)

    def _unbind(self):
        if self.workspace is not None:
            rtdm_unbind_workspace(self.h)
            self.workspace = None

    def close(self):
        if self.h is not None:
            rtdm_destroy(self.h)
            self.h = None
        self.workspace = None
        self.allocator = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def bind_workspace(self, device: int = 0, extra: int = 0):
        """Move the context's device buffers into one torch allocation (kept
        alive by this object), `extra` bytes beyond rtdm_workspace_size's
        figure for calls with large temporaries."""
        import torch
        if self.workspace is not None:
            return self.workspace.numel()
        n = rtdm_workspace_size(self.h) + int(extra)
        self.workspace = torch.empty(n, dtype=torch.uint8, device=f"cuda:{device}")
        rtdm_bind_workspace(self.h, self.workspace.data_ptr(), n)
        return n

    def load_batch(self, systems, kicks, stream=None):
        """One geometry holding every (system, kick) pair as its own group.

        systems: generated systems with equal b and ranges; kicks[k]: the kick
        vectors of systems[k].  Replicas are laid out along x with gaps wider
        than every range, so the matrices are block-diagonal over groups.
        Returns the group pointer.  The kicks are applied by rtdm_apply_kick_groups.
        """
        s0 = systems[0]
        gap = 2.0 * max(s0.R_HS, s0.R_K, s0.R_P) + 1.0
        xyz, rows, cols = [], {"S": [], "H0": [], "K": []}, {"S": [], "H0": [], "K": []}
        data = {"S": [], "H0": [], "K": []}
        gptr, kap = [0], []
        x0 = 0.0
        n = 0
        for sys_, ks in zip(systems, kicks):
            assert sys_.b == s0.b and (sys_.R_HS, sys_.R_K, sys_.R_P) == (s0.R_HS, s0.R_K, s0.R_P)
            for k in ks:
                shift = np.array([x0 - sys_.xyz[:, 0].min(), 0.0, 0.0])
                xyz.append(sys_.xyz + shift)
                x0 += np.ptp(sys_.xyz[:, 0]) + gap
                for name, m in (("S", sys_.S), ("H0", sys_.H0), ("K", sys_.K0)):
                    rows[name].append(m.rows + n)
                    cols[name].append(m.cols + n)
                    data[name].append(m.data)
                n += sys_.n_atoms
                gptr.append(n)
                kap.append(k)
        self.b = s0.b
        xyz = np.concatenate(xyz)
        self._unbind()
        rtdm_set_geometry(self.h, xyz, np.full(n, s0.b, dtype=np.int32))
        rtdm_set_ranges(self.h, s0.R_HS, s0.R_P, s0.R_K)
        rtdm_set_groups(self.h, gptr)
        for name in ("S", "H0", "K"):
            rtdm_upload_coo(self.h, name, np.concatenate(rows[name]), np.concatenate(cols[name]),
                            np.concatenate(data[name]), stream)
        self.batch_xyz = xyz
        self.group_ptr = np.asarray(gptr)
        self.group_kicks = np.asarray(kap, dtype=np.float64)
        return self.group_ptr

    def load_kick_sets(self, systems, kicks, stream=None):
        """One geometry holding each system once as its own group, for a context
        created with n_kicks = len(kicks): kick set k propagates every system
        after the kick kicks[k] (applied by rtdm_apply_kicks with
        self.kick_vectors), all sets sharing one propagator per step.
        Returns the group pointer."""
        assert self.options.n_kicks == len(kicks)
        gptr = self.load_batch(systems, [[(0.0, 0.0, 0.0)]] * len(systems), stream)
        self.kick_vectors = np.asarray(kicks, dtype=np.float64)
        return gptr

    def load_mixed(self, sys_, stream=None):
        """A system with per-atom block sizes (synth.MixedSystem)."""
        self.b = int(sys_.nbf.max())
        self._unbind()
        rtdm_set_geometry(self.h, sys_.xyz, sys_.nbf)
        rtdm_set_ranges(self.h, sys_.R_HS, sys_.R_P, sys_.R_K)
        for name, m in (("S", sys_.S), ("H0", sys_.H0), ("K", sys_.K0)):
            rtdm_upload_coo(self.h, name, m.rows, m.cols, m.data, stream)
        return self

    def load_system(self, sys_, stream=None):
        self.b = sys_.b
        self._unbind()
        rtdm_set_geometry(self.h, sys_.xyz, sys_.nbf)
        rtdm_set_ranges(self.h, sys_.R_HS, sys_.R_P, sys_.R_K)
        for name, m in (("S", sys_.S), ("H0", sys_.H0), ("K", sys_.K0)):
            rtdm_upload_coo(self.h, name, m.rows, m.cols, m.data, stream)
        return self

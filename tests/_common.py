"""Shared helpers of the GPU parity tests (no test functions here)."""

import numpy as np

from oracle import oracle as O
from paper_1404_5776_amd import rtdm

# FP64 parity bar: relative Frobenius error of every compared matrix and
# max-norm error of every trace relative to its scale.
TOL = 1e-10


def rel(a, b) -> float:
    na = np.linalg.norm(np.asarray(b).ravel())
    return float(np.linalg.norm((np.asarray(a) - np.asarray(b)).ravel()) / (na if na > 0 else 1.0))


def gpu_context(sys_, **opts) -> rtdm.Context:
    print(f"[gpu] {sys_.name} b={sys_.b} R_HS={sys_.R_HS} R_P={sys_.R_P} R_K={sys_.R_K} opts={opts}", flush=True)
    return rtdm.Context(0, **opts).load_system(sys_)


def assert_same_pattern(ctx, slot, pat: O.Pattern):
    rp, col = rtdm.rtdm_pattern(ctx.h, slot)
    np.testing.assert_array_equal(rp, pat.row_ptr)
    np.testing.assert_array_equal(col, pat.col)


def dipole_floor(q: np.ndarray, xyz: np.ndarray) -> float:
    """Rounding floor of P = -sum_i (r_i - r_c) q_i: the sum nearly cancels, so
    two FP64 implementations summing in different orders agree only to about
    log2(n) * eps * sum_i |r_i - r_c| |q_i| (forward error of a tree-order sum).
    The centroid r_c is itself a sum with error up to log2(n) * eps * |r_c|,
    and that error is multiplied by the total charge sum_i q_i."""
    rc = xyz.mean(axis=0)
    S = np.abs((xyz - rc) * q[:, None]).sum(axis=0) + np.abs(rc) * abs(q.sum())
    return 2.0 * np.log2(max(len(q), 2)) * np.finfo(float).eps * S.max()

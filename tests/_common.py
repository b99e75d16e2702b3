"""Shared helpers of the GPU parity tests (no test functions here)."""

import numpy as np

from oracle import oracle as O
from paper_1404_5776_amd import rtdm, synth

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


def dipole_floor(q: np.ndarray, xyz: np.ndarray, dq: float = 0.0) -> float:
    """Rounding floor of P = -sum_i (r_i - r_c) q_i between two FP64 codes.

    The sum nearly cancels, so two implementations summing in different
    orders agree only to about log2(n) * eps * sum_i |r_i - r_c| |q_i| (forward
    error of a tree-order sum).  The centroid r_c is the same number in both
    (each coordinate sum rounded once), so it adds no term.  The charges
    themselves differ by rounding (dq = max_i |q_i - q_ref_i|, measured by
    assert_charges on the last step and doubled for the steps before it),
    which moves P by at most dq * sum_i |r_i - r_c|."""
    rc = O.centroid(xyz)
    d = np.abs(xyz - rc)
    S = np.abs(d * q[:, None]).sum(axis=0)
    return 2.0 * np.log2(max(len(q), 2)) * np.finfo(float).eps * S.max() + 2.0 * dq * d.sum(axis=0).max()


def gpu_charges(ctx, n_atoms: int) -> np.ndarray:
    """The context's current Mulliken charges q_i (rtdm_get_state)."""
    return rtdm.rtdm_get_state(ctx.h, n_atoms)[2:2 + n_atoms]


def assert_charges(q: np.ndarray, K_ref: "O.BSM", S: "O.BSM") -> float:
    """Per-atom charges against the oracle's q_i = Re sum_j tr(K_ij S_ji) of its
    K: max |q - q_ref| <= TOL * max |q_ref| (the charges do not cancel, so
    this bar has no rounding floor).  Returns max |q - q_ref|."""
    want = O.mulliken(K_ref, S)
    dq = float(np.abs(q - want).max())
    err = dq / float(np.abs(want).max())
    print(f"charges: max rel error {err:.2e}")
    assert err <= TOL, err
    return dq


def small_clusters(b):
    """Three b = 4 clusters (ranges 8 / 12 bohr) or two b = 13 clusters (6 / 8 bohr)."""
    out = []
    sizes, ranges = ((30, 55, 41), (8.0, 12.0)) if b == 4 else ((24, 37), (6.0, 8.0))
    for k, n in enumerate(sizes):
        xyz = synth.cluster_positions(n, np.random.default_rng(91 + k))
        out.append(synth.build_system(f"c{n}_b{b}", xyz, b, ranges[0], ranges[1], 95 + k, k0="exact"))
    return out


def padded_system(ms, b=13):
    """A mixed-size system (synth.MixedSystem) as an equal-size system of b
    functions per atom: identity in S on each atom's padded functions, zeros
    in H0 and K0 there (the representation the library stores)."""
    def pad(c, eye):
        data = np.zeros((c.nnzb, b, b))
        at = 0
        for t, (i, j) in enumerate(zip(c.rows, c.cols)):
            ni, nj = ms.nbf[i], ms.nbf[j]
            data[t, :ni, :nj] = c.data[at:at + ni * nj].reshape(ni, nj)
            if eye and i == j:
                data[t, ni:, ni:] = np.eye(b - ni)
            at += ni * nj
        return synth.BlockCOO(c.rows, c.cols, data)

    return synth.System(name="padded", xyz=ms.xyz, b=b, R_HS=ms.R_HS, R_K=ms.R_K, R_P=ms.R_P,
                        S=pad(ms.S, True), H0=pad(ms.H0, False), K0=pad(ms.K0, False))


def strip_padding(Kb: "O.BSM", ms) -> np.ndarray:
    """Dense matrix over the real functions from padded blocks."""
    off = np.concatenate([[0], np.cumsum(ms.nbf)])
    out = np.zeros((off[-1], off[-1]), dtype=Kb.val.dtype)
    r = Kb.pat.rows()
    for p in range(Kb.pat.nnzb):
        i, j = int(r[p]), int(Kb.pat.col[p])
        out[off[i]:off[i + 1], off[j]:off[j + 1]] = Kb.val[p, :ms.nbf[i], :ms.nbf[j]]
    return out

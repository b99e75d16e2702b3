"""A(theta) of the Mulliken model formed as A0 + X D (A0 = P_P(X H0), D the
diagonal on-site term) against the full product P_P(X H) at every time point
(option xh_every_step = 1).

The two are equal in exact arithmetic, so their runs agree to rounding
(1e-12 relative here, a hundred times inside the 1e-10 oracle bar that the
parity tests hold both to).  A0 must follow X and H0: after H0 or X is
replaced between calls, a stale A0 would keep the old Hamiltonian and part
the two runs by the size of the change (a percent here); a field switched
off after some steps moves the run from the full product to A0 + X D.  Each
check runs eager and with captured graphs (on the b = 13 path the graph
also reads the column-major copy of X, which must follow a new X).
"""

import numpy as np
import pytest

from paper_1404_5776_amd import rtdm, synth
from tests._common import gpu_context, rel

pytestmark = pytest.mark.gpu

AGREE = 1e-12


def _systems():
    return {
        "b13": synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=31, k0="local", h_model="mulliken"),
        "b4": synth.diamond_lattice((3, 3, 3), 4, 10.0, 12.0, seed=32, h_model="mulliken"),
    }


def _run(s, xh, use_graph, change):
    ctx = gpu_context(s, h_model="mulliken", xh_every_step=xh, use_graph=use_graph, graph_steps=2)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    if change == "field":          # a pulse for the first steps (both runs take the full product then)
        rtdm.rtdm_set_field(ctx.h, (0.002, -0.001, 0.0), 0.1, 0.05)
    rtdm.rtdm_step(ctx.h, s.dt, 4)
    if change == "field":
        rtdm.rtdm_set_field(ctx.h, (0.0, 0.0, 0.0), 0.1, 0.05)
    elif change == "H0":
        rtdm.rtdm_upload_coo(ctx.h, "H0", s.H0.rows, s.H0.cols, 1.01 * s.H0.data)
    elif change == "X":
        X = rtdm.rtdm_download(ctx.h, "X", s.b).real
        rtdm.rtdm_upload(ctx.h, "X", 0.99 * X)
    elif change == "inverse":
        rtdm.rtdm_upload_coo(ctx.h, "S", s.S.rows, s.S.cols, 1.01 * s.S.data)
        rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_step(ctx.h, s.dt, 5)
    out = rtdm.rtdm_download(ctx.h, "K", s.b), rtdm.rtdm_dipole_trace(ctx.h)
    ctx.close()
    return out


@pytest.mark.parametrize("change", ["none", "H0", "X", "inverse", "field"])
@pytest.mark.parametrize("which", ["b13", "b4"])
@pytest.mark.parametrize("use_graph", [0, 1])
def test_a0_path_equals_full_product(which, change, use_graph):
    s = _systems()[which]
    K0, tr0 = _run(s, 1, use_graph, change)
    K1, tr1 = _run(s, 0, use_graph, change)
    e = rel(K1, K0)
    induced = np.abs(tr0[:, 1:4] - tr0[0, 1:4]).max()
    de = np.abs(tr1[:, 1:4] - tr0[:, 1:4]).max()
    print(f"{which} {change} graph={use_graph}: K rel {e:.2e}, dipole {de:.2e} of induced {induced:.2e}")
    assert e <= AGREE
    assert de <= 1e-9 * induced
    assert np.abs(tr1[:, 4] - tr0[:, 4]).max() <= AGREE * np.abs(tr0[:, 4]).max()


def test_changes_reach_the_propagation():
    """The checks above would pass vacuously if the changes did nothing: each
    one moves K by far more than the agreement bar."""
    s = _systems()["b4"]
    K, _ = _run(s, 0, 0, "none")
    for change in ("H0", "X", "inverse", "field"):
        Kc, _ = _run(s, 0, 0, change)
        assert rel(Kc, K) > 1e3 * AGREE, change


def test_xh_every_step_takes_zero_or_one():
    with pytest.raises(rtdm.RtdmError):
        rtdm.Context(0, h_model="mulliken", xh_every_step=2)

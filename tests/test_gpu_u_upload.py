"""A propagator given to the context: after U is uploaded, steps with a fixed
H use it as it is (no rebuild while dt is unchanged), together with the
copies of U that the step products read (the column-major copy on the b = 13
path, U^dagger stored as a matrix for W U^dagger on the b = 4 path).

Run A steps 3 times with dt 0.05, uploads the propagator of dt 0.03 (taken
from another context) and steps 3 more times with dt 0.05: the uploaded U
is kept.  Run B steps 3 times with dt 0.05 and 3 times with dt 0.03, which
rebuilds the same U bit for bit.  Both apply the same products to the same
K, so K and the charges agree bit for bit; a copy of U left from before the
upload would propagate the last 3 steps with the old U.
"""

import numpy as np
import pytest

from paper_1404_5776_amd import rtdm, synth
from tests._common import gpu_charges, gpu_context, rel

pytestmark = pytest.mark.gpu


def _systems():
    return {
        "b13": synth.diamond_lattice((2, 2, 2), 13, 10.0, 16.0, seed=41, k0="local", h_model="fixed"),
        "b4": synth.diamond_lattice((6, 6, 6), 4, 10.0, 12.0, seed=42, h_model="fixed"),
    }


def _start(s, use_graph):
    ctx = gpu_context(s, h_model="fixed", use_graph=use_graph, graph_steps=2)
    rtdm.rtdm_build_inverse(ctx.h)
    rtdm.rtdm_apply_kick(ctx.h, s.kappa)
    return ctx


@pytest.mark.parametrize("use_graph", [0, 1])
@pytest.mark.parametrize("which", ["b13", "b4"])
def test_uploaded_propagator_is_used_with_its_copies(which, use_graph):
    s = _systems()[which]
    donor = _start(s, 0)
    rtdm.rtdm_step(donor.h, 0.03, 1)
    U03 = rtdm.rtdm_download(donor.h, "U", s.b)
    donor.close()

    a = _start(s, use_graph)
    rtdm.rtdm_step(a.h, 0.05, 3)
    U05 = rtdm.rtdm_download(a.h, "U", s.b)
    rtdm.rtdm_upload(a.h, "U", U03)
    rtdm.rtdm_step(a.h, 0.05, 3)
    Ka, qa = rtdm.rtdm_download(a.h, "K", s.b), gpu_charges(a, s.n_atoms)
    a.close()

    b = _start(s, use_graph)
    rtdm.rtdm_step(b.h, 0.05, 3)
    rtdm.rtdm_step(b.h, 0.03, 3)
    Kb, qb = rtdm.rtdm_download(b.h, "K", s.b), gpu_charges(b, s.n_atoms)
    b.close()

    assert rel(U03, U05) > 1e-3          # the upload changes the propagator
    assert np.array_equal(Ka, Kb)
    assert np.array_equal(qa, qb)

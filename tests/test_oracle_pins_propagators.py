"""Pins of the oracle's ETRS and fourth-order Magnus propagators, the
self-consistent (predictor-corrector) midpoint Hamiltonian, the Gaussian
field and the spectrum transform.

References that do not come from the oracle: an adaptive high-order ODE
integration (scipy's DOP853) of the dense Liouville equation
i dK/dt = S^-1 H K - K H S^-1 (Sec. II.A), closed-form orders of accuracy,
exact time reversibility of the symmetric schemes, the exact kick that an
impulsive field produces in an orthonormal basis, and the geometric-series
closed form of the damped transform.
"""

import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

from oracle import oracle as O
from paper_1404_5776_amd import synth

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _tiny(n=6, b=2, seed=4, spread=5.0):
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(0, spread, size=(n, 3))
    s = synth.build_system("tiny", xyz, b, 30.0, 30.0, seed, k0="exact")   # ranges cover everything
    st = O.setup(s)
    return s, st, O.hotelling(st.S, st.pat_p, tol=1e-14)


def _dense_model(st):
    """Dense S, H0, per-function atom positions (relative to the centroid)."""
    S = st.S.to_dense().real
    H0 = st.H0.to_dense().real
    pos = np.repeat(st.xyz - st.xyz.mean(axis=0), st.b, axis=0)
    return S, H0, pos


def _reference(st, T, field=None, gain=0.0, kappa=(0.0, 0.0, 0.0)):
    """K(T) by DOP853 on the dense Liouville equation, H(t, K) written out here."""
    S, H0, pos = _dense_model(st)
    Si = np.linalg.inv(S)
    nb = S.shape[0]
    # position matrices of the dipole reading: (r_a + r_b)/2 S_ab per component
    R = [0.5 * (pos[:, c][:, None] + pos[:, c][None, :]) * S for c in range(3)]
    K0 = O.kick(st.K0, st.xyz, kappa).to_dense()
    atom = np.repeat(np.arange(st.xyz.shape[0]), st.b)
    q_of = lambda K: np.bincount(atom, weights=np.real(np.diag(K @ S)))
    q_ref = q_of(st.K0.to_dense())

    def rhs(t, y):
        K = y.reshape(nb, nb)
        H = H0.copy()
        if gain:
            H = H + np.diag(gain * (q_of(K) - q_ref)[atom])
        if field is not None:
            E = field.at(t)
            H = H + sum(E[c] * R[c] for c in range(3))
        A = Si @ H
        return (-1j * (A @ K - K @ A.conj().T)).ravel()

    sol = solve_ivp(rhs, (0.0, T), K0.ravel().astype(complex), method="DOP853", rtol=1e-12, atol=1e-14)
    return sol.y[:, -1].reshape(nb, nb)


FIELD = O.Field((0.6, -0.3, 0.2), 0.8, 0.3)


@pytest.mark.parametrize("kind,order", [("em", 2), ("etrs", 2), ("m4", 4)])
def test_order_with_time_dependent_field(kind, order):
    """Explicitly time-dependent H = H0 - E(t).r: EM and ETRS are second order,
    the Gauss-Legendre Magnus propagator fourth order."""
    s, st, inv = _tiny()
    T = 1.6
    ref = _reference(st, T, field=FIELD)

    def final(dt):
        n = int(round(T / dt))
        return O.propagate(st, n, dt, (0, 0, 0), p=14, X=inv, propagator=kind, field=FIELD).K.to_dense()

    e = [np.abs(final(dt) - ref).max() for dt in (0.2, 0.1, 0.05)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert all(order - 0.3 < o < order + 0.5 for o in orders), (e, orders)


@pytest.mark.parametrize("kind", ["em", "etrs", "m4"])
def test_impulsive_field_in_orthonormal_basis_is_the_kick(kind):
    """With S = I and H0 = 0 the field term is E(t).diag(r - r_c); all its values
    commute, so the propagation over the pulse is exactly the phase
    exp(i kappa.(r_i - r_j)) on K_ij with kappa = -integral of E (the kick), up
    to the quadrature of that integral by the step's time points."""
    rng = np.random.default_rng(7)
    xyz = rng.uniform(0, 6, size=(5, 3))
    b = 2
    pat = O.pattern(xyz, 30.0)
    S = O.identity(pat, b)
    H0 = O.zeros(pat, b)
    Kd = rng.normal(size=(10, 10)) + 1j * rng.normal(size=(10, 10))
    Kd = Kd + Kd.conj().T
    K0 = O.BSM(pat, b, np.stack([Kd[2 * i:2 * i + 2, 2 * j:2 * j + 2]
                                 for i, j in zip(pat.rows(), pat.col)]))
    st = O.Setup(xyz, b, pat, pat, pat, S, H0, K0)
    sigma, t0 = 0.25, 2.5
    kappa = np.array([0.3, -0.2, 0.1])
    field = O.Field(tuple(-kappa / (sigma * math.sqrt(2 * math.pi))), t0, sigma)
    dt, n = 0.02, 250
    K = O.propagate(st, n, dt, (0, 0, 0), p=14, propagator=kind, field=field).K
    want = O.kick(K0, xyz, kappa)
    assert np.abs(K.val - want.val).max() < 1e-9 * np.abs(want.val).max()


@pytest.mark.parametrize("kind", ["em", "etrs", "m4"])
def test_time_points_of_each_scheme(kind):
    """S = I, H0 = 0 and a coarse step: the accumulated phase is exactly the
    quadrature of the field by each scheme's own time points, midpoint (EM),
    trapezoid (ETRS) and two-point Gauss-Legendre (M4)."""
    rng = np.random.default_rng(8)
    xyz = rng.uniform(0, 6, size=(4, 3))
    b = 1
    pat = O.pattern(xyz, 30.0)
    Kd = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    Kd = Kd + Kd.conj().T
    K0 = O.BSM(pat, b, np.array([[[Kd[i, j]]] for i, j in zip(pat.rows(), pat.col)]))
    st = O.Setup(xyz, b, pat, pat, pat, O.identity(pat, b), O.zeros(pat, b), K0)
    f = O.Field((0.4, -0.3, 0.2), 0.35, 0.2)
    dt, n = 0.25, 6
    nodes = {"em": [(0.5, 1.0)], "etrs": [(0.0, 0.5), (1.0, 0.5)],
             "m4": [(O.M4_THETA[0], 0.5), (O.M4_THETA[1], 0.5)]}[kind]
    integral = sum(w * dt * f.at((k + th) * dt) for k in range(n) for th, w in nodes)
    K = O.propagate(st, n, dt, (0, 0, 0), p=30, propagator=kind, field=f).K
    want = O.kick(K0, xyz, -integral)
    assert np.abs(K.val - want.val).max() < 1e-12 * np.abs(want.val).max()


@pytest.mark.parametrize("kind", ["em", "etrs", "m4"])
def test_symmetric_schemes_are_time_reversible_with_field(kind):
    """Forward n steps, then n steps with -dt from the end time, returns K0."""
    s, st, inv = _tiny(seed=5)
    n, dt = 12, 0.1
    fwd = O.propagate(st, n, dt, (0, 0, 0), p=16, X=inv, propagator=kind, field=FIELD)
    st2 = O.Setup(st.xyz, st.b, st.pat_hs, st.pat_p, st.pat_k, st.S, st.H0, fwd.K)
    back = O.propagate(st2, n, -dt, (0, 0, 0), p=16, X=inv, propagator=kind, field=FIELD, t_start=n * dt)
    assert np.abs(back.K.val - st.K0.val).max() < 1e-12


@pytest.mark.parametrize("kind", ["em", "etrs", "m4"])
def test_self_consistent_step_is_time_reversible_and_converged(kind):
    """With H(K), the corrector iterated to convergence makes the charges at
    each time point the interpolation between q(t) and q(t + dt), which is
    time reversible; the extrapolating predictor alone is not."""
    s, st, inv = _tiny(seed=6)
    g = 4.0
    q_ref = O.mulliken(st.K0, st.S)
    n, dt = 8, 0.1
    kappa = (0.8, 0.0, 0.0)

    def there_and_back(sc_iters):
        kw = dict(h_model="mulliken", h_gain=g, p=16, X=inv, sc_steps=n, sc_iters=sc_iters, q_ref=q_ref,
                  propagator=kind)
        fwd = O.propagate(st, n, dt, kappa, **kw)
        st2 = O.Setup(st.xyz, st.b, st.pat_hs, st.pat_p, st.pat_k, st.S, st.H0, fwd.K)
        back = O.propagate(st2, n, -dt, (0, 0, 0), t_start=n * dt, **kw)
        return fwd.K, np.abs(back.K.val - O.kick(st.K0, st.xyz, kappa).val).max()

    K20, err20 = there_and_back(20)
    K40, _ = there_and_back(40)
    _, err0 = there_and_back(0)
    assert np.abs(K20.val - K40.val).max() < 1e-13          # the corrector has converged
    assert err20 < 1e-11                                      # reversible at the fixed point
    assert err0 > 1e3 * err20                                 # the predictor alone is not


@pytest.mark.parametrize("sc", [0, 3])
def test_mulliken_h_second_order_with_and_without_corrector(sc):
    s, st, inv = _tiny(seed=8)
    T, kappa, g = 1.6, (0.8, 0.0, 0.0), 4.0
    ref = _reference(st, T, gain=g, kappa=kappa)

    def final(dt):
        n = int(round(T / dt))
        return O.propagate(st, n, dt, kappa, h_model="mulliken", h_gain=g, p=14, X=inv,
                           sc_steps=n if sc else 0, sc_iters=sc).K.to_dense()

    e = [np.abs(final(dt) - ref).max() for dt in (0.2, 0.1, 0.05)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert all(1.7 < o < 2.4 for o in orders), (e, orders)


def test_m4_with_constant_h_is_the_plain_exponential():
    """A(t) constant: the commutator vanishes and M = -i dt A exactly."""
    s = synth.config1()
    st = O.setup(s)
    inv = O.hotelling(st.S, st.pat_p)
    a = O.propagate(st, 3, 0.05, s.kappa, X=inv)
    b = O.propagate(st, 3, 0.05, s.kappa, X=inv, propagator="m4")
    assert np.abs(a.K.val - b.K.val).max() < 1e-15 * np.abs(a.K.val).max() * 100


def _dense_a(st, S, H0, pos, t=None, field=None, q=None, gain=0.0, q_ref=None):
    """S^-1 H for the dense model, H written out here (field and on-site shift)."""
    H = H0.copy()
    if field is not None:
        E = field.at(t)
        H = H + sum(E[c] * 0.5 * (pos[:, c][:, None] + pos[:, c][None, :]) * S for c in range(3))
    if q is not None:
        H = H + np.diag(np.repeat(gain * (q - q_ref), st.b))
    return np.linalg.solve(S, H)


def _dense_u(kind, a_at, dt):
    if kind == "em":
        return expm(-1j * dt * a_at(0.5))
    if kind == "etrs":
        return expm(-0.5j * dt * a_at(1.0)) @ expm(-0.5j * dt * a_at(0.0))
    t1, t2 = 0.5 - math.sqrt(3) / 6, 0.5 + math.sqrt(3) / 6
    A1, A2 = a_at(t1), a_at(t2)
    return expm(-0.5j * dt * (A1 + A2) - math.sqrt(3) * dt * dt / 12 * (A2 @ A1 - A1 @ A2))


@pytest.mark.parametrize("kind", ["em", "etrs", "m4"])
def test_one_step_equals_dense_matrix_exponential(kind):
    """One untruncated step with a time-dependent field against the scheme's
    formula evaluated with scipy's expm on dense matrices."""
    s, st, inv = _tiny(seed=10)
    S, H0, pos = _dense_model(st)
    dt, t0 = 0.3, 0.55
    U = _dense_u(kind, lambda th: _dense_a(st, S, H0, pos, t0 + th * dt, FIELD), dt)
    K0 = st.K0.to_dense()
    want = U @ K0 @ U.conj().T
    got = O.propagate(st, 1, dt, (0, 0, 0), p=30, X=inv, propagator=kind, field=FIELD, t_start=t0).K.to_dense()
    assert np.abs(got - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("kind", ["em", "etrs", "m4"])
def test_converged_corrector_satisfies_the_step_equation(kind):
    """After the corrector has converged, K1 = U(q0, q1) K0 U(q0, q1)^dagger with
    the charges at each of the scheme's time points interpolated linearly
    between q0 = q(K0) and q1 = q(K1), checked with dense expm."""
    s, st, inv = _tiny(seed=11)
    S, H0, pos = _dense_model(st)
    g, dt = 4.0, 0.15
    atom = np.repeat(np.arange(st.xyz.shape[0]), st.b)
    q_of = lambda K: np.bincount(atom, weights=np.real(np.diag(K @ S)))
    q_ref = q_of(st.K0.to_dense())
    kappa = (0.6, -0.2, 0.0)
    K0 = O.kick(st.K0, st.xyz, kappa).to_dense()
    K1 = O.propagate(st, 1, dt, kappa, h_model="mulliken", h_gain=g, p=30, X=inv, propagator=kind,
                     sc_steps=1, sc_iters=60).K.to_dense()
    q0, q1 = q_of(K0), q_of(K1)
    U = _dense_u(kind, lambda th: _dense_a(st, S, H0, pos, q=q0 + th * (q1 - q0), gain=g, q_ref=q_ref), dt)
    want = U @ K0 @ U.conj().T
    assert np.abs(K1 - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("kind", ["em", "etrs", "m4"])
def test_predictor_extrapolates_charges_to_each_time_point(kind):
    """Second step without corrector: K2 = U K1 U^dagger with the charges at
    each time point extrapolated from q(t - dt) = q(K0) and q(t) = q(K1)."""
    s, st, inv = _tiny(seed=12)
    S, H0, pos = _dense_model(st)
    g, dt = 4.0, 0.15
    atom = np.repeat(np.arange(st.xyz.shape[0]), st.b)
    q_of = lambda K: np.bincount(atom, weights=np.real(np.diag(K @ S)))
    q_ref = q_of(st.K0.to_dense())
    kappa = (0.6, -0.2, 0.0)
    kw = dict(h_model="mulliken", h_gain=g, p=30, X=inv, propagator=kind)
    K0 = O.kick(st.K0, st.xyz, kappa).to_dense()
    K1 = O.propagate(st, 1, dt, kappa, **kw).K.to_dense()
    K2 = O.propagate(st, 2, dt, kappa, **kw).K.to_dense()
    q0, q1 = q_of(K0), q_of(K1)
    U = _dense_u(kind, lambda th: _dense_a(st, S, H0, pos, q=q1 + th * (q1 - q0), gain=g, q_ref=q_ref), dt)
    want = U @ K1 @ U.conj().T
    assert np.abs(K2 - want).max() < 1e-12 * np.abs(want).max()


# ------------------------------------------------------------------ spectra

def test_damped_transform_matches_geometric_series():
    dt, n, w0, gamma = 0.05, 400, 1.3, 0.2
    t = dt * np.arange(1, n + 1)
    a = np.array([0.7, -0.2, 0.0])
    P0 = np.array([1.0, 2.0, 3.0])
    P = P0[None, :] + np.sin(w0 * t)[:, None] * a[None, :]
    om = np.linspace(0.1, 3.0, 30)
    kappa = np.array([0.5, 0.25, 0.0])
    alpha, Sw = O.spectrum(P, P0, dt, None, kappa, gamma, om)

    def geo(z):   # sum_{k=0}^{n} exp(z k)
        return (1 - np.exp(z * (n + 1))) / (1 - np.exp(z))

    F = (geo((1j * (om + w0) - gamma) * dt) - geo((1j * (om - w0) - gamma) * dt)) / (2j) * dt
    np.testing.assert_allclose(alpha[:, 0], -a[0] * F / kappa[0], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(alpha[:, 1], -a[1] * F / kappa[1], rtol=1e-12, atol=1e-14)
    assert np.all(np.isnan(alpha[:, 2]))
    np.testing.assert_allclose(Sw, 2 * om / np.pi * np.imag((alpha[:, 0] + alpha[:, 1]) / 3))


def test_kicked_dimer_absorbs_at_its_excitation_energy():
    """Two sites: the strength function peaks at the excitation energy, with a
    positive sign (absorption), which ties the kick, dipole and transform signs."""
    e, t, s_ = -0.2, -0.3, 0.25
    xyz = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0]])
    pat = O.pattern(xyz, 5.0)
    S = O.BSM(pat, 1, np.array([[[1.0]], [[s_]], [[s_]], [[1.0]]], dtype=complex))
    H = O.BSM(pat, 1, np.array([[[e]], [[t]], [[t]], [[e]]], dtype=complex))
    c = 1.0 / math.sqrt(2 * (1 + s_))
    K0 = O.BSM(pat, 1, np.full((4, 1, 1), c * c, dtype=complex))
    st = O.Setup(xyz, 1, pat, pat, pat, S, H, K0)
    dt, n, kap = 0.05, 2000, 1e-3
    tr = O.propagate(st, n, dt, (kap, 0.0, 0.0), p=5, inv_tol=1e-14)
    P0 = O.dipole(O.mulliken(O.kick(K0, xyz, (kap, 0, 0)), S), xyz)
    om = np.linspace(0.05, 2.0, 400)
    _, Sw = O.spectrum(tr.rows[:, 1:4], P0, dt, None, np.array([kap, 0, 0]), 0.02, om)
    omega = abs((e - t) / (1 - s_) - (e + t) / (1 + s_))
    k = np.argmax(np.abs(Sw))
    assert Sw[k] > 0
    assert abs(om[k] - omega) <= 2 * (om[1] - om[0]) + 2 * math.pi / (n * dt)


def test_polarisability_does_not_depend_on_the_pulse_shape():
    """Linear response: two weak Gaussian pulses of different width, centre and
    strength give the same alpha(w) where both have spectral weight."""
    s, st, inv = _tiny(seed=9)
    dt, n, gamma = 0.05, 600, 0.1
    om = np.linspace(0.2, 2.0, 19)
    P0 = O.dipole(O.mulliken(st.K0, st.S), st.xyz)
    out = []
    for amp, sigma, t0 in ((2e-4, 0.1, 0.5), (-1e-4, 0.15, 0.8)):
        f = O.Field((amp, 0.5 * amp, 0.0), t0, sigma)
        tr = O.propagate(st, n, dt, (0, 0, 0), p=8, X=inv, field=f)
        E = np.array([f.at(k * dt) for k in range(n + 1)])
        a, _ = O.spectrum(tr.rows[:, 1:4], P0, dt, E, None, gamma, om)
        assert np.all(np.isnan(a[:, 2]))
        out.append(a[:, :2])
    np.testing.assert_allclose(out[0], out[1], rtol=1e-3, atol=1e-3 * np.abs(out[1]).max())

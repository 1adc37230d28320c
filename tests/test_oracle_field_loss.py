"""Pins of the oracle's time-dependent external field, its loss and the
absolute normalisation of its exchange energy.

The field profile follows the reading of the paper's input record
``-externfield Hx Hy Hz startTime decayTime stopTime`` (Sec. 5): off before
startTime, full strength up to decayTime, linear decay to zero at stopTime,
off afterwards.  A one-cell sample in a field of fixed direction and
magnitude s(t) H follows the static-field LLG trajectory in the rescaled
time I(t) = integral of s, so the macrospin closed form with I(t) in place of
t pins the profile's shape and end points.  The exchange energy of a lattice
helix has a closed form that fixes its prefactor A V / d^2 absolutely (the
field is tied to the energy by the finite-difference pin in
test_oracle_pins.py).
"""
import math

import numpy as np
import pytest

import oracle
from tests.closed_forms import macrospin

GAMMA0 = 2.211e5


def _macrospin_problem(Hz, alpha):
    return oracle.Problem((1, 1, 1), (5e-9,) * 3, alpha=alpha, hext=(0, 0, Hz), terms=oracle.T_ZEEMAN)


def _m0(th0=1.0, ph0=0.3):
    return np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)]).reshape(3, 1, 1, 1)


def test_constant_schedule_equals_constant_field_run():
    """A schedule that is on for the whole run reproduces the plain run bit
    for bit (all four terms, a 4x3x2 sample)."""
    rng = np.random.default_rng(2)
    n, d = (4, 3, 2), (5e-9, 4e-9, 3e-9)
    P = oracle.Problem(n, d, Ms=8e5, A=1.3e-11, Ku=2e4, u=(0.0, 0.6, 0.8), alpha=0.2,
                       hext=rng.standard_normal((3, 2, 3, 4)) * 2e4)
    m0 = rng.standard_normal((3, 2, 3, 4))
    m0 /= np.linalg.norm(m0, axis=0)
    ref = P.run(m0, 30, 1e-13)
    got, t = P.run_scheduled(m0, 30, 1e-13, (-1.0, 1.0, 2.0))
    np.testing.assert_array_equal(got, ref)
    assert t == sum([1e-13] * 30)


def test_field_is_off_before_start_and_after_stop():
    """Zeeman field only: before startTime and after stopTime the state does
    not move at all."""
    P = _macrospin_problem(1e5, 0.1)
    m0 = _m0()
    m, t = P.run_scheduled(m0, 100, 1e-13, (5e-11, 6e-11, 7e-11))
    np.testing.assert_array_equal(m, m0)
    m1, t1 = P.run_scheduled(m0, 800, 1e-13, (0.0, 2e-11, 4e-11))
    m2, _ = P.run_scheduled(m1, 300, 1e-13, (0.0, 2e-11, 4e-11), t0=t1)
    np.testing.assert_array_equal(m2, m1)
    assert np.abs(m1 - m0).max() > 0.1


@pytest.mark.parametrize("sched", [(2e-11, 8e-11, 1.5e-10), (0.0, 1e-10, 1e-10), (3e-11, 3e-11, 1.7e-10)])
def test_macrospin_follows_rescaled_time(sched):
    """One spin, field H z-hat times the profile: the exact solution is the
    static-field one at I(T) = (t_decay - t_start) + (t_stop - t_decay)/2
    (T past t_stop).  Euler at dt = 1e-15 s is within 2e-4 of it; the
    profile read as a step at t_decay or at t_stop instead would be O(1)
    off."""
    alpha, Hz, T, dt = 0.1, 1e5, 2e-10, 1e-15
    ts, td, tp = sched
    P = _macrospin_problem(Hz, alpha)
    m, t = P.run_scheduled(_m0(), int(round(T / dt)), dt, sched)
    I = (td - ts) + 0.5 * (tp - td)
    exact = macrospin(1.0, 0.3, Hz, alpha, GAMMA0, I)
    err = np.linalg.norm(m.ravel() - exact)
    assert err < 2e-4, err
    for wrong in (td - ts, tp - ts):
        if abs(wrong - I) > 1e-12:
            assert np.linalg.norm(macrospin(1.0, 0.3, Hz, alpha, GAMMA0, wrong) - exact) > 100 * err


def test_field_scale_integral_by_quadrature():
    """The profile integrates to (t_decay - t_start) + (t_stop - t_decay)/2
    (midpoint rule on a fine grid, independent of the oracle's run loop)."""
    sched = (1e-11, 4e-11, 9e-11)
    h = 1e-14
    ts = (np.arange(20000) + 0.5) * h
    total = math.fsum(oracle.field_scale(t, sched) for t in ts) * h
    assert abs(total - (3e-11 + 2.5e-11)) < 1e-16


def test_loss_special_cases():
    """1/2 sum |m - t|^2: zero for m = t; N for orthogonal unit fields;
    2N for opposite unit fields; exact fsum on a random case."""
    rng = np.random.default_rng(4)
    N = 1000
    m = rng.standard_normal((3, N))
    m /= np.linalg.norm(m, axis=0)
    assert oracle.loss(m, m) == 0.0
    x = np.zeros((3, N)); x[0] = 1.0
    y = np.zeros((3, N)); y[1] = 1.0
    assert oracle.loss(x, y) == N
    assert abs(oracle.loss(m, -m) - 2 * N) < 1e-10
    t = rng.standard_normal((3, N))
    exact = 0.5 * math.fsum(float(v) for v in ((m - t) ** 2).ravel())
    assert abs(oracle.loss(m, t) - exact) < 1e-12 * exact


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_exchange_energy_of_a_lattice_helix(axis):
    """m rotating by k d per cell along one axis: every neighbour pair along
    that axis has |m_j - m_i|^2 = 2 - 2 cos(k d), pairs along the other axes
    none, so E_ex = A V (pairs) (2 - 2 cos(k d)) / d^2 exactly."""
    n, d = (7, 5, 4), (4e-9, 5e-9, 3e-9)
    A = 1.3e-11
    k = 0.37 / d[axis]
    nx, ny, nz = n
    idx = np.indices((nz, ny, nx))[[2, 1, 0][axis]]  # cell index along `axis`
    phase = k * idx * d[axis]
    m = np.stack([np.cos(phase), np.sin(phase), np.zeros_like(phase)])
    P = oracle.Problem(n, d, Ms=8e5, A=A, terms=oracle.T_EXCH)
    E = P.energy(m)[0]
    pairs = (n[axis] - 1) * (nx * ny * nz // n[axis])
    V = d[0] * d[1] * d[2]
    exact = A * V * pairs * (2 - 2 * math.cos(k * d[axis])) / d[axis] ** 2
    assert abs(E - exact) < 1e-12 * exact, (E, exact)

"""Pins of the FP64 oracle against things other than itself.

Each test ties one part of the oracle to a closed form, an exact identity, an
independent evaluation or a convergence law, chosen so that a plausible slip
(a dropped term, a wrong sign or index, a transposed operand) fails.

Paper: Zhu, arXiv:1411.2565.  Sec. 2 eq. (1) energy, eq. (2) effective field,
eq. (3) LLG; Sec. 3 FFT demag convolution (exactly the direct sum pinned
here), six-neighbour exchange, explicit Euler.
"""
import itertools

import numpy as np
import pytest

import oracle
from tests.closed_forms import aharoni, dipole_tensor, macrospin

MU0 = oracle.MU0


# ---------------------------------------------------------------- tensor --

@pytest.mark.parametrize("d", [(5e-9, 5e-9, 5e-9), (4e-9, 4e-9, 3e-9), (1e-9, 2e-9, 7e-9)])
def test_self_term_equals_aharoni_prism(d):
    """N(0) of one cell is the prism demag factor (Aharoni closed form)."""
    N = oracle.tensor_at(0, 0, 0, *d)
    np.testing.assert_allclose(N[:3], aharoni(*d), rtol=0, atol=1e-12)
    assert abs(N[:3].sum() - 1.0) < 1e-13
    assert np.abs(N[3:]).max() < 1e-14


def test_cube_self_term_is_one_third():
    N = oracle.tensor_at(0, 0, 0, 5e-9, 5e-9, 5e-9)
    np.testing.assert_allclose(N[:3], 1 / 3, atol=1e-14)


OFFSETS = [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (2, 1, 3), (5, 4, 2), (11, 3, 7),
           (13, 0, 0), (20, 9, 4), (40, 33, 17)]


@pytest.mark.parametrize("o", OFFSETS)
@pytest.mark.parametrize("d", [(5e-9, 5e-9, 5e-9), (4e-9, 4e-9, 3e-9)])
def test_trace_vanishes_off_centre(o, d):
    """The dipole kernel is harmonic away from the source: trace N(o) = 0."""
    N = oracle.tensor_at(o[0] * d[0], o[1] * d[1], o[2] * d[2], *d)
    assert abs(N[:3].sum()) < 1e-12


@pytest.mark.parametrize("o", [(2, 1, 3), (5, 4, 2), (14, 3, 2)])
def test_parities(o):
    """Diagonal components are even in every axis; xy is odd in x and y and
    even in z (likewise xz, yz)."""
    d = (4e-9, 4e-9, 3e-9)
    base = oracle.tensor_at(o[0] * d[0], o[1] * d[1], o[2] * d[2], *d)
    for s in itertools.product([1, -1], repeat=3):
        N = oracle.tensor_at(s[0] * o[0] * d[0], s[1] * o[1] * d[1], s[2] * o[2] * d[2], *d)
        # absolute bound: the 27-point sums round differently at mirrored points
        tol = dict(rtol=0, atol=1e-14)
        np.testing.assert_allclose(N[:3], base[:3], **tol)
        np.testing.assert_allclose(N[3], s[0] * s[1] * base[3], **tol)
        np.testing.assert_allclose(N[4], s[0] * s[2] * base[4], **tol)
        np.testing.assert_allclose(N[5], s[1] * s[2] * base[5], **tol)
        assert abs(base[3]) > 1e-6 and abs(base[4]) > 1e-6 and abs(base[5]) > 1e-6


def test_far_field_dipole_limit_and_order():
    """N(r) -> (V/4 pi)(I - 3 rr^T)/r^3 with error O((d/r)^4) for cubes."""
    d = 5e-9
    V = d ** 3
    errs = []
    for k in (4, 8, 16):
        o = np.array([3, 2, 1]) * k / 4
        r = o * d
        N = oracle.tensor_at(*r, d, d, d)
        D = dipole_tensor(r, V)
        errs.append(np.abs(N - D).max() / np.abs(D).max())
    # error ratio between r and 2r close to 16
    assert errs[2] < 1e-5
    for a, b in zip(errs, errs[1:]):
        assert 10 < a / b < 24, errs


@pytest.mark.parametrize("o", [(6, 4, 2), (8, 6, 3), (12, 8, 5), (16, 11, 6)])
def test_newell_agrees_with_tent_quadrature(o):
    """Two independent evaluations of the same cell-pair integral."""
    d = (4e-9, 4e-9, 3e-9)
    r = [o[i] * d[i] for i in range(3)]
    a = oracle.tensor_at(*r, *d, method=1)
    b = oracle.tensor_at(*r, *d, method=2, nodes=8)
    assert np.abs(a - b).max() < 1e-9 * 0.4


def test_table_layout_matches_pointwise():
    n, d = (5, 4, 3), (4e-9, 4e-9, 3e-9)
    tab = oracle.tensor_table(n, d)
    for (ox, oy, oz) in [(0, 0, 0), (4, 3, 2), (1, 2, 0), (3, 0, 1)]:
        np.testing.assert_allclose(tab[:, oz, oy, ox],
                                   oracle.tensor_at(ox * d[0], oy * d[1], oz * d[2], *d), rtol=1e-14)


# ------------------------------------------------------------ demag sum --

@pytest.mark.parametrize("n,d", [((16, 16, 2), (5e-9,) * 3), ((4, 3, 2), (5e-9,) * 3),
                                 ((32, 8, 1), (4e-9, 4e-9, 3e-9)), ((7, 5, 3), (2e-9, 3e-9, 4e-9))])
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_uniform_body_average_equals_aharoni(n, d, axis):
    """For uniform M, the cell average of H_d is -D_body Ms e (Aharoni factors
    of the whole sample): exact for cell-averaged tensors."""
    P = oracle.Problem(n, d, Ms=8e5)
    m = np.zeros((3, n[2], n[1], n[0]))
    m[axis] = 1.0
    Hbar = P.demag(m).mean(axis=(1, 2, 3))
    Db = aharoni(n[0] * d[0], n[1] * d[1], n[2] * d[2])
    expect = np.zeros(3)
    expect[axis] = -Db[axis] * 8e5
    np.testing.assert_allclose(Hbar, expect, rtol=0, atol=8e5 * 2e-11)


def test_direct_sum_brute_force_with_signed_offsets():
    """Loop organisation and parity signs of the fast direct sum against a
    pure-Python double loop that evaluates N at the signed offset."""
    n, d = (3, 2, 2), (4e-9, 3e-9, 5e-9)
    rng = np.random.default_rng(3)
    m = rng.standard_normal((3, 2, 2, 3))
    Ms = 8e5 * (0.5 + rng.random((2, 2, 3)))
    P = oracle.Problem(n, d, Ms=Ms)
    H = P.demag(m)
    cells = list(itertools.product(range(2), range(2), range(3)))
    Hb = np.zeros_like(m)
    for (iz, iy, ix) in cells:
        for (jz, jy, jx) in cells:
            t = oracle.tensor_at((ix - jx) * d[0], (iy - jy) * d[1], (iz - jz) * d[2], *d)
            N = np.array([[t[0], t[3], t[4]], [t[3], t[1], t[5]], [t[4], t[5], t[2]]])
            Hb[:, iz, iy, ix] -= N @ (Ms[jz, jy, jx] * m[:, jz, jy, jx])
    np.testing.assert_allclose(H, Hb, rtol=1e-12, atol=1e-9)


def test_single_source_far_field_sign():
    """A lone magnetised cell seen from far away is a point dipole:
    H = (1/4 pi) (3 r(r.m) - m r^2) Ms V / r^5, which fixes the sign of the
    off-diagonal components along a diagonal offset."""
    n, d = (24, 24, 1), (5e-9,) * 3
    Ms = np.zeros((1, 24, 24))
    Ms[0, 0, 0] = 8e5
    P = oracle.Problem(n, d, Ms=Ms)
    m = np.zeros((3, 1, 24, 24))
    m[0] = 1.0
    H = P.demag(m)[:, 0, 23, 23]
    r = np.array([23, 23, 0]) * 5e-9
    rr = np.linalg.norm(r)
    mm = np.array([8e5, 0, 0])
    Hd = (3 * r * (r @ mm) - mm * rr ** 2) * (5e-9) ** 3 / (4 * np.pi * rr ** 5)
    np.testing.assert_allclose(H, Hd, rtol=1e-4, atol=1e-12 * np.abs(Hd).max())
    assert H[1] > 0


def test_observer_subset_matches_full():
    n, d = (9, 7, 3), (5e-9,) * 3
    rng = np.random.default_rng(5)
    m = rng.standard_normal((3, 3, 7, 9))
    P = oracle.Problem(n, d, Ms=8.6e5)
    H = P.demag(m).reshape(3, -1)
    obs = np.array([0, 5, 17, 60, 188])
    np.testing.assert_allclose(P.demag_observers(m, obs), H[:, obs], rtol=1e-13, atol=1e-9)


def test_step_cells_equals_full_step_at_those_cells():
    n, d = (9, 6, 3), (4e-9, 4e-9, 3e-9)
    rng = np.random.default_rng(21)
    m = rng.standard_normal((3, 3, 6, 9))
    m /= np.linalg.norm(m, axis=0)
    P = oracle.Problem(n, d, Ms=8e5 * (0.6 + rng.random((3, 6, 9))), Ku=2e4, u=(0, 0.6, 0.8),
                       hext=rng.standard_normal((3, 3, 6, 9)) * 1e4, alpha=0.2)
    cells = np.array([0, 8, 9, 53, 100, 161])
    full = P.run(m, 1, 3e-14).reshape(3, -1)[:, cells]
    np.testing.assert_allclose(P.step_cells(m, cells, 3e-14), full, rtol=1e-12, atol=1e-14)


def test_convolution_is_self_adjoint():
    n, d = (6, 5, 3), (4e-9, 4e-9, 3e-9)
    tab = oracle.tensor_table(n, d)
    rng = np.random.default_rng(7)
    a, b = rng.standard_normal((2, 3, 3, 5, 6))
    lhs = np.sum(a * oracle.conv(n, tab, b))
    rhs = np.sum(oracle.conv(n, tab, a) * b)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# -------------------------------------------------------------- exchange --

def test_exchange_uniform_is_zero():
    n, d = (8, 6, 4), (5e-9,) * 3
    m = np.zeros((3, 4, 6, 8))
    m[1] = 1.0
    P = oracle.Problem(n, d, terms=oracle.T_EXCH)
    assert np.abs(P.heff(m)).max() == 0.0


@pytest.mark.parametrize("axis,p", [(0, 1), (0, 3), (1, 2), (2, 1)])
def test_exchange_neumann_cosine_eigenmode(axis, p):
    """cos(pi p (i+1/2)/n) is an eigenvector of the free-boundary six-neighbour
    Laplacian with eigenvalue -(4/d^2) sin^2(pi p / (2 n))."""
    n, d = (10, 8, 6), (4e-9, 3e-9, 5e-9)
    shape = (n[2], n[1], n[0])
    idx = np.indices(shape)[2 - axis]
    mode = np.cos(np.pi * p * (idx + 0.5) / n[axis])
    m = np.zeros((3,) + shape)
    m[2] = mode
    Ms, A = 7e5, 1.1e-11
    P = oracle.Problem(n, d, Ms=Ms, A=A, terms=oracle.T_EXCH)
    lam = -(4 / d[axis] ** 2) * np.sin(np.pi * p / (2 * n[axis])) ** 2
    H = P.heff(m)
    np.testing.assert_allclose(H[2], 2 * A / (MU0 * Ms) * lam * mode, rtol=1e-12, atol=1e-3)
    assert np.abs(H[:2]).max() == 0.0


def test_laplacian_symmetric():
    n, d = (5, 4, 3), (4e-9, 3e-9, 5e-9)
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal((2, 3, 3, 4, 5))
    lhs = np.sum(a * oracle.laplacian(n, d, b))
    rhs = np.sum(oracle.laplacian(n, d, a) * b)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# --------------------------------------------------- anisotropy / Zeeman --

def test_anisotropy_closed_forms():
    n, d = (3, 2, 1), (5e-9,) * 3
    u = np.array([1.0, 2.0, 2.0]) / 3.0
    Ms, Ku = 8e5, 5e2
    P = oracle.Problem(n, d, Ms=Ms, Ku=Ku, u=tuple(u), terms=oracle.T_ANIS)
    m = np.broadcast_to(u[:, None, None, None], (3, 1, 2, 3)).copy()
    HK = 2 * Ku / (MU0 * Ms)
    np.testing.assert_allclose(P.heff(m), HK * m, rtol=1e-13)
    perp = np.cross(u, [0.0, 0.0, 1.0])
    perp /= np.linalg.norm(perp)
    m = np.broadcast_to(perp[:, None, None, None], (3, 1, 2, 3)).copy()
    assert np.abs(P.heff(m)).max() < 1e-10 * HK


def test_zeeman_is_identity():
    n, d = (3, 2, 2), (5e-9,) * 3
    rng = np.random.default_rng(2)
    h = rng.standard_normal((3, 2, 2, 3)) * 1e4
    P = oracle.Problem(n, d, hext=h, terms=oracle.T_ZEEMAN)
    m = rng.standard_normal((3, 2, 2, 3))
    np.testing.assert_array_equal(P.heff(m), h)


# ------------------------------------------------------------------ LLG --

def test_llg_fixed_point_and_orthogonality():
    n, d = (4, 3, 2), (5e-9,) * 3
    rng = np.random.default_rng(4)
    P = oracle.Problem(n, d, alpha=0.3)
    m = rng.standard_normal((3, 2, 3, 4))
    m /= np.linalg.norm(m, axis=0)
    H = 1e5 * m * rng.random((1, 2, 3, 4))
    assert np.abs(P.llg_rhs(m, H)).max() < 1e-6   # m || H
    H = rng.standard_normal((3, 2, 3, 4)) * 1e5
    f = P.llg_rhs(m, H)
    assert np.abs(np.sum(f * m, axis=0)).max() < 1e-6 * np.abs(f).max()


def test_llg_precession_sense_and_rate():
    """m = x, H = H z: dm/dt = gamma0 H/(1+a^2) (y + a z-ish).  Explicitly
    f = c1 m x H + c2 m x (m x H) with c1 = -gamma0/(1+a^2), c2 = a c1."""
    P = oracle.Problem((1, 1, 1), (5e-9,) * 3, alpha=0.2)
    m = np.array([1.0, 0, 0]).reshape(3, 1, 1, 1)
    H = np.array([0, 0, 2e4]).reshape(3, 1, 1, 1)
    f = P.llg_rhs(m, H).ravel()
    w = 2.211e5 * 2e4 / (1 + 0.04)
    np.testing.assert_allclose(f, [0.0, w, 0.2 * w], rtol=1e-13)


def test_macrospin_euler_converges_first_order():
    """One cell in a static field: Euler + renormalisation approaches the
    exact LLG solution with error halving as dt halves."""
    alpha, Hz, T = 0.1, 1e5, 0.2e-9
    th0, ph0 = 1.0, 0.3
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)])
    P = oracle.Problem((1, 1, 1), (5e-9,) * 3, alpha=alpha, hext=(0, 0, Hz), terms=oracle.T_ZEEMAN)
    exact = macrospin(th0, ph0, Hz, alpha, 2.211e5, T)
    errs = []
    for dt in (1e-13, 5e-14, 2.5e-14):
        m = P.run(m0.reshape(3, 1, 1, 1), int(round(T / dt)), dt).ravel()
        errs.append(np.linalg.norm(m - exact))
    assert errs[0] < 5e-3
    for a, b in zip(errs, errs[1:]):
        assert 1.8 < a / b < 2.2, errs


@pytest.mark.parametrize("method,dts,ratio", [("heun", (4e-13, 2e-13, 1e-13), 4.0),
                                              ("rk4", (2e-12, 1e-12, 5e-13), 16.0)])
def test_macrospin_runge_kutta_orders(method, dts, ratio):
    """Heun (order 2) and classic Runge-Kutta (order 4) on the exact
    macrospin solution: the error falls by 2^order as dt halves."""
    alpha, Hz, T = 0.1, 1e5, 0.2e-9
    th0, ph0 = 1.0, 0.3
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)])
    P = oracle.Problem((1, 1, 1), (5e-9,) * 3, alpha=alpha, hext=(0, 0, Hz), terms=oracle.T_ZEEMAN)
    exact = macrospin(th0, ph0, Hz, alpha, 2.211e5, T)
    errs = [np.linalg.norm(P.run(m0.reshape(3, 1, 1, 1), int(round(T / dt)), dt, method=method).ravel() - exact)
            for dt in dts]
    for a, b in zip(errs, errs[1:]):
        assert 0.9 * ratio < a / b < 1.1 * ratio, errs


def _coupled_problem():
    rng = np.random.default_rng(3)
    m = rng.standard_normal((3, 2, 3, 4))
    m /= np.linalg.norm(m, axis=0)
    P = oracle.Problem((4, 3, 2), (5e-9,) * 3, Ms=8e5, A=1.3e-11, Ku=3e4, u=(0.6, 0.0, 0.8), alpha=0.5,
                       hext=(1e4, -2e4, 5e3))
    return P, m


@pytest.mark.parametrize("method,base,ratio", [("heun", 4e-14, 4.0), ("rk4", 8e-14, 16.0)])
def test_runge_kutta_orders_with_all_terms(method, base, ratio):
    """The same orders on a 4x3x2 sample with demag, exchange, anisotropy and
    Zeeman terms (reference: the same method at dt/32).  A wrong tableau
    entry would drop the order to one."""
    P, m = _coupled_problem()
    T = 4e-12
    ref = P.run(m, int(round(T / (base / 32))), base / 32, method=method)
    errs = [np.linalg.norm(P.run(m, int(round(T / dt)), dt, method=method) - ref)
            for dt in (base, base / 2, base / 4)]
    for a, b in zip(errs, errs[1:]):
        assert 0.9 * ratio < a / b < 1.15 * ratio, errs


def test_runge_kutta_methods_integrate_the_same_equation():
    """Euler, Heun and RK4 at small steps reach the same state (they differ
    only in truncation error), so the higher-order steps use the same f."""
    P, m = _coupled_problem()
    T = 4e-12
    rk4 = P.run(m, 200, T / 200, method="rk4")
    heun = P.run(m, 1600, T / 1600, method="heun")
    euler = P.run(m, 12800, T / 12800)
    scale = np.linalg.norm(rk4 - m)
    assert np.linalg.norm(heun - rk4) < 1e-5 * scale
    assert np.linalg.norm(euler - rk4) < 5e-3 * scale
    for pair in ("heun_euler", "bs23", "dp54"):  # adaptive pairs at a tight tolerance
        ma = P.run_adaptive(m, T, 1e-14, 1e-8, pair)[0]
        assert np.linalg.norm(ma - rk4) < 1e-6 * scale, pair


def _macrospin_setup(T=0.2e-9):
    alpha, Hz = 0.1, 1e5
    th0, ph0 = 1.0, 0.3
    m0 = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)]).reshape(3, 1, 1, 1)
    P = oracle.Problem((1, 1, 1), (5e-9,) * 3, alpha=alpha, hext=(0, 0, Hz), terms=oracle.T_ZEEMAN)
    return P, m0, T, macrospin(th0, ph0, Hz, alpha, 2.211e5, T)


@pytest.mark.parametrize("pair,T,steps_ratio", [("heun_euler", 0.2e-9, 10.0),
                                                ("bs23", 0.2e-9, 100.0 ** (1 / 3)),
                                                ("dp54", 1e-9, 100.0 ** (1 / 5))])
def test_adaptive_pairs_scale_with_tolerance(pair, T, steps_ratio):
    """Adaptive steps on the exact macrospin solution: the global error is
    proportional to the tolerance, and the number of accepted steps grows as
    tol^(-1/(q+1)) (q the lower order: 1 for Heun/Euler, 2 for
    Bogacki-Shampine, 4 for Dormand-Prince, whose few large steps need the
    longer horizon).  A wrong weight in either member of the pair changes
    one of the two exponents."""
    P, m0, T, exact = _macrospin_setup(T)
    res = {tol: P.run_adaptive(m0, T, 1e-13, tol, pair) for tol in (1e-5, 1e-7)}
    err = {tol: np.linalg.norm(r[0].ravel() - exact) for tol, r in res.items()}
    assert 70 < err[1e-5] / err[1e-7] < 140, err
    assert err[1e-7] < 1e-6
    ratio = res[1e-7][2] / res[1e-5][2]
    assert 0.8 * steps_ratio < ratio < 1.25 * steps_ratio, (res[1e-5][2], res[1e-7][2])


def test_heun_euler_estimate_is_the_difference_of_the_two_steps():
    """Without renormalisation the error estimate of the 2(1) pair after one
    step equals max over cells |Heun step - Euler step|, computed here from
    the oracle's separate Euler and Heun steps; it is read back from the
    proposed next step dt' = dt 0.9 (tol/err)^(1/2)."""
    rng = np.random.default_rng(12)
    m = rng.standard_normal((3, 2, 3, 4))
    m /= np.linalg.norm(m, axis=0)
    P = oracle.Problem((4, 3, 2), (5e-9,) * 3, Ms=8e5, A=1.3e-11, alpha=0.3, hext=(1e4, 0, 0), renorm=False)
    dt = 2e-14
    diff = P.run(m, 1, dt, method="heun") - P.run(m, 1, dt)
    err = np.linalg.norm(diff, axis=0).max()
    tol = 2.0 * err
    m1, dt_next, acc, rej = P.run_adaptive(m, dt, dt, tol, "heun_euler")
    assert (acc, rej) == (1, 0)
    np.testing.assert_allclose(m1, P.run(m, 1, dt, method="heun"), rtol=0, atol=1e-15)
    implied = tol * (0.9 * dt / dt_next) ** 2
    np.testing.assert_allclose(implied, err, rtol=1e-9)


def test_norm_identity_without_renorm():
    """f is orthogonal to m, so |m + dt f|^2 = |m|^2 + dt^2 |f|^2 exactly."""
    n, d = (6, 5, 2), (5e-9,) * 3
    rng = np.random.default_rng(8)
    m = rng.standard_normal((3, 2, 5, 6))
    m /= np.linalg.norm(m, axis=0)
    P = oracle.Problem(n, d, alpha=0.5, renorm=False)
    dt = 1e-13
    f = P.llg_rhs(m, P.heff(m))
    m1 = P.run(m, 1, dt)
    lhs = np.sum(m1 ** 2, axis=0)
    rhs = 1.0 + dt ** 2 * np.sum(f ** 2, axis=0)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13)
    assert np.abs(lhs - 1).max() > 1e-8  # the dt^2 term is really there


# --------------------------------------------------------------- energy --

def test_field_is_minus_energy_gradient():
    """H_i = -(1/(mu0 Ms_i V)) dE/dm_i for every term (finite differences of
    the energy of eq. (1) against the field of eq. (2))."""
    n, d = (4, 3, 2), (4e-9, 5e-9, 3e-9)
    rng = np.random.default_rng(9)
    Ms = 8e5 * (0.7 + 0.6 * rng.random((2, 3, 4)))
    h = rng.standard_normal((3, 2, 3, 4)) * 3e4
    u = np.array([0.6, 0.0, 0.8])
    P = oracle.Problem(n, d, Ms=Ms, Ku=3e4, u=tuple(u), hext=h, A=1.3e-11)
    m = rng.standard_normal((3, 2, 3, 4))
    H = P.heff(m)
    V = d[0] * d[1] * d[2]
    eps = 1e-6
    for c, iz, iy, ix in [(0, 0, 0, 0), (1, 1, 2, 3), (2, 1, 1, 2), (0, 0, 2, 1)]:
        mp, mm = m.copy(), m.copy()
        mp[c, iz, iy, ix] += eps
        mm[c, iz, iy, ix] -= eps
        g = (P.energy(mp)[4] - P.energy(mm)[4]) / (2 * eps)
        np.testing.assert_allclose(-g / (MU0 * Ms[iz, iy, ix] * V), H[c, iz, iy, ix], rtol=1e-6)


def test_energy_decreases_with_damping():
    n, d = (8, 8, 2), (5e-9,) * 3
    rng = np.random.default_rng(0)
    m = rng.standard_normal((3, 2, 8, 8))
    m /= np.linalg.norm(m, axis=0)
    P = oracle.Problem(n, d, alpha=0.5, Ku=2e4, u=(0, 0, 1.0), hext=(1e4, 0, 0))
    E = [P.energy(m)[4]]
    for _ in range(40):
        m = P.run(m, 1, 2e-14)
        E.append(P.energy(m)[4])
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-12 * np.abs(E[:-1]))
    assert E[-1] < E[0]


def test_energy_drift_is_first_order_without_damping():
    """alpha = 0: Euler's energy drift over a fixed time halves with dt."""
    n, d = (6, 6, 2), (5e-9,) * 3
    rng = np.random.default_rng(11)
    m0 = rng.standard_normal((3, 2, 6, 6))
    m0 /= np.linalg.norm(m0, axis=0)
    P = oracle.Problem(n, d, alpha=0.0)
    E0 = P.energy(m0)[4]
    T = 2e-12
    drifts = []
    for dt in (4e-15, 2e-15, 1e-15):
        m = P.run(m0, int(round(T / dt)), dt)
        drifts.append(abs(P.energy(m)[4] - E0))
    for a, b in zip(drifts, drifts[1:]):
        assert 1.7 < a / b < 2.3, drifts


# -------------------------------------------------------------- adjoint --

def _problem_for_grad(renorm=True):
    n, d = (4, 3, 2), (5e-9, 5e-9, 5e-9)
    rng = np.random.default_rng(12)
    Ms = 8e5 * (0.8 + 0.4 * rng.random((2, 3, 4)))
    h = rng.standard_normal((3, 2, 3, 4)) * 2e4
    m0 = rng.standard_normal((3, 2, 3, 4))
    m0 /= np.linalg.norm(m0, axis=0)
    t = rng.standard_normal((3, 2, 3, 4))
    t /= np.linalg.norm(t, axis=0)
    kw = dict(A=1.3e-11, Ku=4e4, u=(0.0, 0.6, 0.8), alpha=0.3, renorm=renorm)
    return n, d, Ms, h, m0, t, kw


@pytest.mark.parametrize("renorm", [True, False])
def test_adjoint_matches_central_differences(renorm):
    n, d, Ms, h, m0, t, kw = _problem_for_grad(renorm)
    steps, dt = 6, 2e-14
    P = oracle.Problem(n, d, Ms=Ms, hext=h, **kw)
    loss, gm, gh, gms = P.adjoint(m0, steps, dt, t)

    def L(m0_=m0, h_=h, Ms_=Ms):
        Q = oracle.Problem(n, d, Ms=Ms_, hext=h_, tab=P.tab, **kw)
        mT = Q.run(m0_, steps, dt)
        return 0.5 * np.sum((mT - t) ** 2)

    assert abs(L() - loss) < 1e-14 * max(1.0, loss)
    rng = np.random.default_rng(13)
    # step sizes where central-difference truncation (O(e^2)) and rollout
    # rounding (~1e-15/e) are both below 1e-7 relative; the FD error was
    # seen to fall as e^2 toward the adjoint value
    for _ in range(3):
        v = rng.standard_normal(m0.shape)
        e = 1e-5
        fd = (L(m0_=m0 + e * v) - L(m0_=m0 - e * v)) / (2 * e)
        np.testing.assert_allclose(np.sum(gm * v), fd, rtol=1e-7, atol=1e-14)
        v = rng.standard_normal(h.shape) * 2e4
        e = 1e-3
        fd = (L(h_=h + e * v) - L(h_=h - e * v)) / (2 * e)
        np.testing.assert_allclose(np.sum(gh * v), fd, rtol=1e-7, atol=1e-14)
        v = rng.standard_normal(Ms.shape) * 8e5
        e = 1e-5
        fd = (L(Ms_=Ms + e * v) - L(Ms_=Ms - e * v)) / (2 * e)
        np.testing.assert_allclose(np.sum(gms * v), fd, rtol=1e-7, atol=1e-14)


# ------------------------------------------------- non-regular geometry --

def _padded_pair():
    """A 5x4x2 sample with Ms, field and state maps, and the same sample
    embedded at offset (2, 1, 1) in a 9x7x4 grid whose other cells are
    vacuum (Ms = 0) holding arbitrary m and field values."""
    rng = np.random.default_rng(4)
    n0, n1, off, d = (5, 4, 2), (9, 7, 4), (2, 1, 1), (4e-9, 5e-9, 3e-9)
    sl = (Ellipsis, slice(off[2], off[2] + n0[2]), slice(off[1], off[1] + n0[1]), slice(off[0], off[0] + n0[0]))
    m0 = rng.standard_normal((3, n0[2], n0[1], n0[0]))
    m0 /= np.linalg.norm(m0, axis=0)
    ms0 = 8e5 * (0.8 + 0.4 * rng.random((n0[2], n0[1], n0[0])))
    h0 = 2e4 * rng.standard_normal((3, n0[2], n0[1], n0[0]))
    m1 = rng.standard_normal((3, n1[2], n1[1], n1[0]))
    m1 /= np.linalg.norm(m1, axis=0)
    m1[sl] = m0
    ms1 = np.zeros((n1[2], n1[1], n1[0]))
    ms1[sl] = ms0
    h1 = np.full((3, n1[2], n1[1], n1[0]), 3e4)
    h1[sl] = h0
    kw = dict(A=1.3e-11, Ku=3e4, u=(0.6, 0.0, 0.8), alpha=0.3)
    P0 = oracle.Problem(n0, d, Ms=ms0, hext=h0, **kw)
    P1 = oracle.Problem(n1, d, Ms=ms1, hext=h1, **kw)
    return P0, P1, m0, m1, sl, ms1 > 0


def test_vacuum_padding_is_invisible():
    """Vacuum cells are no demag source, cut exchange like a free surface and
    do not move: padding a sample with vacuum leaves its fields, trajectory
    (Euler and adaptive) and energies unchanged, and the vacuum cells'
    state untouched."""
    P0, P1, m0, m1, sl, mag = _padded_pair()
    np.testing.assert_allclose(P1.heff(m1)[sl], P0.heff(m0), rtol=0, atol=1e-9)
    r0, r1 = P0.run(m0, 20, 2e-14), P1.run(m1, 20, 2e-14)
    np.testing.assert_allclose(r1[sl], r0, rtol=0, atol=1e-13)
    assert np.array_equal(r1[:, ~mag], m1[:, ~mag])
    np.testing.assert_allclose(P1.energy(m1), P0.energy(m0), rtol=1e-12)
    a0 = P0.run_adaptive(m0, 5e-13, 1e-14, 1e-5, "bs23")
    a1 = P1.run_adaptive(m1, 5e-13, 1e-14, 1e-5, "bs23")
    assert a0[2:] == a1[2:]
    np.testing.assert_allclose(a1[0][sl], a0[0], rtol=0, atol=1e-13)


def test_vacuum_cells_have_only_stray_and_applied_fields():
    """In vacuum the exchange and anisotropy fields vanish; the demag (stray)
    field and the applied field remain."""
    P0, P1, m0, m1, sl, mag = _padded_pair()
    H = P1.heff(m1, oracle.T_EXCH | oracle.T_ANIS)
    assert np.all(H[:, ~mag] == 0)
    Hd = P1.heff(m1, oracle.T_DEMAG)
    assert np.abs(Hd[:, ~mag]).max() > 1e3
    Hz = P1.heff(m1, oracle.T_ZEEMAN)
    np.testing.assert_array_equal(Hz, np.asarray(P1.hext))


def test_cubic_body_average_demag_is_one_third():
    """A body with the symmetry of the cube (here a staircase sphere of
    radius 8 cells cut from a 18^3 grid by the Ms map) has equal average
    demag factors, and they sum to one: uniform M gives a volume-averaged
    field of exactly -M/3 inside."""
    R, N = 8, 18
    c = np.arange(N) + 0.5 - N / 2
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    inside = x * x + y * y + z * z < R * R
    m = np.zeros((3, N, N, N))
    m[2] = 1.0
    P = oracle.Problem((N, N, N), (5e-9,) * 3, Ms=np.where(inside, 8e5, 0.0), A=1.3e-11, terms=oracle.T_DEMAG)
    Hd = P.demag(m)
    assert inside.sum() == 2176
    np.testing.assert_allclose(Hd[2][inside].mean() / 8e5, -1.0 / 3.0, rtol=1e-10)
    assert abs(Hd[0][inside].mean()) < 1e-10 * 8e5


def test_ms_map_must_be_non_negative():
    with pytest.raises(ValueError):
        oracle.Problem((2, 2, 1), (5e-9,) * 3, Ms=np.array([[[1e5, -1.0], [1e5, 1e5]]]))
    P0, P1, m0, m1, sl, mag = _padded_pair()
    with pytest.raises(ValueError):
        P1.adjoint(m1, 2, 1e-14, m1)

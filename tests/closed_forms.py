"""Closed forms from the literature that pin the oracle from outside.

These are independent of the oracle's own formulas: Aharoni's prism demag
factor is a different expression from Newell's cell tensor, the point-dipole
field is the far-field limit, and the macrospin solution is the exact LLG
trajectory in a static field.
"""
import numpy as np


def aharoni_dz(a, b, c):
    """Demag factor along z of a uniformly magnetised prism with sides
    2a x 2b x 2c (Aharoni, J. Appl. Phys. 83, 3432 (1998), eq. 1)."""
    r = np.sqrt(a * a + b * b + c * c)
    rab, rbc, rac = np.sqrt(a * a + b * b), np.sqrt(b * b + c * c), np.sqrt(a * a + c * c)
    v = ((b * b - c * c) / (2 * b * c) * np.log((r - a) / (r + a))
         + (a * a - c * c) / (2 * a * c) * np.log((r - b) / (r + b))
         + b / (2 * c) * np.log((rab + a) / (rab - a))
         + a / (2 * c) * np.log((rab + b) / (rab - b))
         + c / (2 * a) * np.log((rbc - b) / (rbc + b))
         + c / (2 * b) * np.log((rac - a) / (rac + a))
         + 2 * np.arctan(a * b / (c * r))
         + (a ** 3 + b ** 3 - 2 * c ** 3) / (3 * a * b * c)
         + (a * a + b * b - 2 * c * c) * r / (3 * a * b * c)
         + c / (a * b) * (rac + rbc)
         - (rab ** 3 + rbc ** 3 + rac ** 3) / (3 * a * b * c))
    return v / np.pi


def aharoni(lx, ly, lz):
    """(Dx, Dy, Dz) of an lx x ly x lz prism."""
    a, b, c = lx / 2, ly / 2, lz / 2
    return np.array([aharoni_dz(b, c, a), aharoni_dz(c, a, b), aharoni_dz(a, b, c)])


def dipole_tensor(r, V):
    """Point-dipole limit of the cell tensor: (V/4 pi)(I - 3 rhat rhat^T)/|r|^3,
    returned in the order xx, yy, zz, xy, xz, yz."""
    r = np.asarray(r, dtype=float)
    d = np.linalg.norm(r)
    rh = r / d
    M = (np.eye(3) - 3 * np.outer(rh, rh)) * V / (4 * np.pi * d ** 3)
    return np.array([M[0, 0], M[1, 1], M[2, 2], M[0, 1], M[0, 2], M[1, 2]])


def macrospin(theta0, phi0, H, alpha, gamma0, t):
    """Exact LLG solution for one spin in a static field H z-hat:
    tan(theta/2) = tan(theta0/2) exp(-alpha w t), phi = phi0 + w t,
    w = gamma0 H / (1 + alpha^2)."""
    w = gamma0 * H / (1 + alpha ** 2)
    th = 2 * np.arctan(np.tan(theta0 / 2) * np.exp(-alpha * w * t))
    ph = phi0 + w * t
    return np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])

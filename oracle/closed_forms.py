"""Closed forms that pin the oracle to something other than itself.

TEST INFRASTRUCTURE ONLY (see oracle/core.py).

* Born ion: a charge q at the centre of a sphere of radius a (dielectric eps_p
  inside, eps_s and Debye parameter kappa outside).  The paper's analytic
  sphere test (Section 5) is this case.
* Kirkwood sphere: several charges inside the sphere; series over multipole
  degree n with the exterior modified spherical Bessel function k_n.
* Van Oosterom-Strackee signed solid angle of a triangle seen from a point.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import eval_legendre

from .core import COULOMB_KCAL


def born_energy(q, a, eps_p, eps_s, kappa):
    """E = C_e q^2 / (2a) [1/(eps_s (1 + kappa a)) - 1/eps_p]  (kcal/mol)."""
    return COULOMB_KCAL * q * q / (2.0 * a) * (
        1.0 / (eps_s * (1.0 + kappa * a)) - 1.0 / eps_p)


def born_surface_values(q, a, eps_s, kappa):
    """Exact f = phi_ext and h = dphi_ext/dn on the Born sphere, internal units."""
    f = q / (4.0 * math.pi * eps_s * (1.0 + kappa * a) * a)
    h = -q / (4.0 * math.pi * eps_s * a * a)
    return f, h


def _g_n(nmax, x):
    """g_n = x k_n'(x) / k_n(x) for the exponentially decaying modified
    spherical Bessel function k_n (k_0 = e^{-x}/x), n = 0..nmax.
    Uses k_n' = -k_{n-1} - (n+1) k_n / x and the ratio rho_n = k_{n-1}/k_n,
    rho_0 = 1, rho_{n+1} = 1 / (rho_n + (2n+1)/x)."""
    g = np.zeros(nmax + 1)
    if x == 0.0:
        return -(np.arange(nmax + 1) + 1.0)
    rho = 1.0
    for n in range(nmax + 1):
        g[n] = -x * rho - (n + 1.0)
        rho = 1.0 / (rho + (2 * n + 1.0) / x)
    return g


def kirkwood_energy(q, pos, a, eps_p, eps_s, kappa, tol=1e-15, nmax=400):
    """Polar (reaction-field) energy of point charges inside a sphere of
    radius a centred at the origin, kcal/mol."""
    q = np.asarray(q, float)
    pos = np.asarray(pos, float).reshape(-1, 3)
    b = np.linalg.norm(pos, axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        u = pos / np.where(b > 0, b, 1.0)[:, None]
    cosg = np.clip(u @ u.T, -1.0, 1.0)
    bb = np.outer(b, b) / (a * a)
    qq = np.outer(q, q)
    g = _g_n(nmax, kappa * a)
    total = 0.0
    for n in range(nmax + 1):
        fac = (eps_s * g[n] + (n + 1) * eps_p) / (n * eps_p - eps_s * g[n])
        term = (qq * bb ** n * eval_legendre(n, cosg)).sum() * fac / (eps_p * a)
        total += term
        if n > 2 and abs(term) < tol * abs(total) and (bb.max() ** n) < tol:
            break
    return 0.5 * COULOMB_KCAL * total


def solid_angle(p, v0, v1, v2):
    """Signed solid angle of triangle (v0,v1,v2) seen from p (Van Oosterom &
    Strackee 1983): positive when the triangle's CCW normal points away
    from p."""
    a, b, c = (np.asarray(v, float) - np.asarray(p, float) for v in (v0, v1, v2))
    la, lb, lc = (np.linalg.norm(v, axis=-1) for v in (a, b, c))
    num = np.einsum("...i,...i->...", a, np.cross(b, c))
    den = (la * lb * lc + np.einsum("...i,...i->...", a, b) * lc
           + np.einsum("...i,...i->...", a, c) * lb
           + np.einsum("...i,...i->...", b, c) * la)
    return 2.0 * np.arctan2(num, den)

"""Closed-form two-body motion for oracle pins (paper Sec. 5.1).

Independent of the oracle: Lagrange f and g functions with the eccentric
anomaly difference from Kepler's equation solved by Newton iteration.
"""
import math

import numpy as np


def elements(mu, r, v):
    """Energy per unit reduced mass, semi-major axis, angular momentum vector,
    eccentricity and Laplace-Runge-Lenz vector (per unit reduced mass)."""
    rn = np.linalg.norm(r)
    eps = 0.5 * v @ v - mu / rn
    a = -mu / (2.0 * eps)
    h = np.cross(r, v)
    A = np.cross(v, h) - mu * r / rn
    e = np.linalg.norm(A) / mu
    return dict(energy=eps, a=a, h=h, A=A, e=e)


def propagate(mu, r0, v0, dt):
    """Relative state after time dt on the bound Kepler orbit through (r0, v0)."""
    r0 = np.asarray(r0, dtype=float)
    v0 = np.asarray(v0, dtype=float)
    r0n = np.linalg.norm(r0)
    el = elements(mu, r0, v0)
    a = el["a"]
    if not a > 0:
        raise ValueError("unbound orbit")
    n = math.sqrt(mu / a ** 3)
    P = 2.0 * math.pi / n
    k = math.floor(dt / P)
    dtr = dt - k * P
    sig = (r0 @ v0) / math.sqrt(mu)
    sa = math.sqrt(a)
    c1 = 1.0 - r0n / a
    M = n * dtr
    E = M
    for _ in range(100):
        f = E - c1 * math.sin(E) + sig / sa * (1.0 - math.cos(E)) - M
        fp = 1.0 - c1 * math.cos(E) + sig / sa * math.sin(E)
        dE = -f / fp
        E += dE
        if abs(dE) < 1e-16:
            break
    r = a + (r0n - a) * math.cos(E) + sig * sa * math.sin(E)
    f = 1.0 - a / r0n * (1.0 - math.cos(E))
    g = dtr + math.sqrt(a ** 3 / mu) * (math.sin(E) - E)
    fd = -math.sqrt(mu * a) / (r * r0n) * math.sin(E)
    gd = 1.0 - a / r * (1.0 - math.cos(E))
    return f * r0 + g * v0, fd * r0 + gd * v0

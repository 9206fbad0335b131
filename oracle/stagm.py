"""Smooth-truncated amplitude-Gaussian metric (ST-AGM), Sec. 2.2 of the paper.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Per entry, with b = f(j) >= 0 and truncation 0 < eps < 1 (eq. obj-1):
    g(x; b) = (1-eps)/2 * (b - |x|^2/eps)   if |x| < eps*sqrt(b)
            = (|x| - sqrt(b))^2 / 2          otherwise.
Gradient (eq. objgrad): (1 - 1/eps) x inside the cap, (1 - sqrt(b)/|x|) x outside.
Lipschitz constant of the gradient: L = 2/eps - 1 (Lemma 2.1).

Proximal map Prox_{G;lam}(y) = argmin_z G(z) + lam/2 |z - y|^2 (eq. Prox_sol).
The printed branch threshold is garbled; it is read as
    |y| < (eps - (1-eps)/lam) * sqrt(f)
which is the condition that the truncated branch's stationary point lies inside
the cap.  In that branch the magnitude is max(0, lam|y| / (lam - (1-eps)/eps)),
otherwise (sqrt(f) + lam|y|)/(1 + lam); the phase of y is kept, and for y = 0
(every phase minimises) sign(0) is taken as +1.
"""
from __future__ import annotations

import numpy as np


def g_eps(x, b, eps: float):
    """Elementwise ST-AGM g_eps(x; b)."""
    x = np.asarray(x)
    b = np.asarray(b, dtype=np.float64)
    ax = np.abs(x)
    sb = np.sqrt(b)
    inside = ax < eps * sb
    quad = 0.5 * (1.0 - eps) * (b - ax * ax / eps)
    agm = 0.5 * (ax - sb) ** 2
    return np.where(inside, quad, agm)


def G_eps(z, f, eps: float) -> float:
    """G_eps(z; f) = sum_j g_eps(z(j); f(j))."""
    return float(np.sum(g_eps(z, f, eps)))


def grad_g(x, b, eps: float):
    """Gradient of g_eps with respect to (Re x, Im x), returned as a complex number."""
    x = np.asarray(x, dtype=np.complex128)
    b = np.asarray(b, dtype=np.float64)
    ax = np.abs(x)
    sb = np.sqrt(b)
    inside = ax < eps * sb
    safe = np.where(ax > 0, ax, 1.0)
    outside_scale = 1.0 - sb / safe
    return np.where(inside, (1.0 - 1.0 / eps) * x, outside_scale * x)


def lipschitz(eps: float) -> float:
    """L = 2/eps - 1 (Lemma 2.1)."""
    return 2.0 / eps - 1.0


def prox(y, f, eps: float, lam: float):
    """Closed-form Prox_{G_eps; lam}(y) against intensities f (elementwise, complex128)."""
    y = np.asarray(y, dtype=np.complex128)
    sf = np.sqrt(np.asarray(f, dtype=np.float64))
    ay = np.abs(y)
    phase = np.where(ay > 0, y / np.where(ay > 0, ay, 1.0), 1.0 + 0.0j)
    kappa = (1.0 - eps) / eps
    threshold = (eps - (1.0 - eps) / lam) * sf
    trunc = ay < threshold
    if lam > kappa:
        rho_trunc = np.maximum(0.0, lam * ay / (lam - kappa))
    else:
        rho_trunc = np.zeros_like(ay)   # branch unreachable: threshold <= 0
    rho_agm = (sf + lam * ay) / (1.0 + lam)
    rho = np.where(trunc, rho_trunc, rho_agm)
    return phase * rho

"""Amplitude data term and its gradient with respect to the image and the probe.

TEST INFRASTRUCTURE ONLY (see the package docstring).

L(u, w) = sum_j || |X_j| - sqrt(f_j) ||^2 with X_j = F(w o S_j u), F unitary.  This
is twice the AGM data term of Sec. 2.2 (the eps = 0 case of eq. obj-1) summed over
frames.  Gradients follow the real-gradient convention dL/dRe + i dL/dIm:
  g_j   = 2 (1 - sqrt(f_j)/|X_j|) X_j   (0 where X_j = 0)
  dL/du = sum_j S_j^T( conj(w) o F^{-1} g_j )
  dL/dw = sum_j conj(S_j u) o F^{-1} g_j
(the same structure as the whole-domain optimality condition after eq. objgrad).
"""
from __future__ import annotations

import numpy as np

from . import operators as ops


def loss(u, w, offsets, f) -> float:
    X = ops.forward(u, w, offsets)
    return float(np.sum((np.abs(X) - np.sqrt(f)) ** 2))


def grad(u, w, offsets, f):
    """(L, dL/du, dL/dw)."""
    p = w.shape[0]
    X = ops.forward(u, w, offsets)
    aX = np.abs(X)
    sf = np.sqrt(f)
    scale = np.where(aX > 0, 1.0 - sf / np.where(aX > 0, aX, 1.0), 0.0)
    g = 2.0 * scale * X
    phi = ops.ifft2(g)
    gu = np.zeros(u.shape, dtype=np.complex128)
    gw = np.zeros((p, p), dtype=np.complex128)
    for j, off in enumerate(offsets):
        ops.scatter_add(gu, np.conj(w) * phi[j], off)
        gw += np.conj(ops.gather(u, off, p)) * phi[j]
    return float(np.sum((aX - sf) ** 2)), gu, gw

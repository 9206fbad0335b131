"""Measurement operators, written from Sec. 2 of the paper (problem statement and eq. AtA).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* F is the normalized 2-D DFT, read as unitary (orthonormal scaling 1/p for a
  p x p frame) because that is what makes A*A diagonal (eq. AtA).  Forward sign
  exp(-2 pi i k.x / p), index 0 at the zero frequency, no shift.
* S_j extracts the p x p window whose top-left is (row_j, col_j); S_j^T adds a
  p x p patch back at the same place.
* (A u)_j = F(w o S_j u);  A* y = sum_j S_j^T( conj(w) o F^{-1} y_j ).
* A*A = diag( sum_j S_j^T |w|^2 ).
"""
from __future__ import annotations

import numpy as np


def fft2(x: np.ndarray) -> np.ndarray:
    """Unitary forward 2-D DFT over the last two axes."""
    return np.fft.fft2(x, norm="ortho")


def ifft2(x: np.ndarray) -> np.ndarray:
    """Inverse of :func:`fft2` (its adjoint, since it is unitary)."""
    return np.fft.ifft2(x, norm="ortho")


def gather(u: np.ndarray, off, p: int) -> np.ndarray:
    """S_j u: the p x p window of u at top-left off=(row, col)."""
    r, c = int(off[0]), int(off[1])
    return u[r:r + p, c:c + p]


def scatter_add(target: np.ndarray, patch: np.ndarray, off) -> None:
    """target += S_j^T patch (in place)."""
    r, c = int(off[0]), int(off[1])
    p = patch.shape[0]
    target[r:r + p, c:c + p] += patch


def forward(u: np.ndarray, w: np.ndarray, offsets) -> np.ndarray:
    """A u as a stack [J,p,p] (frames in the order of ``offsets``)."""
    p = w.shape[0]
    out = np.empty((len(offsets), p, p), dtype=np.complex128)
    for j, off in enumerate(offsets):
        out[j] = fft2(w * gather(u, off, p))
    return out


def adjoint(frames: np.ndarray, w: np.ndarray, offsets, shape) -> np.ndarray:
    """A* y = sum_j S_j^T(conj(w) o F^{-1} y_j) on an array of the given shape."""
    out = np.zeros(shape, dtype=np.complex128)
    p = w.shape[0]
    for j, off in enumerate(offsets):
        scatter_add(out, np.conj(w) * ifft2(frames[j]), off)
    assert out.shape[0] >= p
    return out


def illumination(w: np.ndarray, offsets, shape) -> np.ndarray:
    """diag(A*A) = sum_j S_j^T |w|^2 (float64)."""
    out = np.zeros(shape, dtype=np.float64)
    a2 = np.abs(w) ** 2
    for off in offsets:
        scatter_add(out, a2, off)
    return out


def intensities(u: np.ndarray, w: np.ndarray, offsets) -> np.ndarray:
    """Noise-free measurements f_j = |F(w o S_j u)|^2 (the forward model of the problem statement)."""
    return np.abs(forward(u, w, offsets)) ** 2

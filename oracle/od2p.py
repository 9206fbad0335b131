"""OD2P / OD2Pm (Algorithms 1 and 2 of the paper), step by step, in complex128.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One iteration n -> n+1 of Algorithm 2 (Algorithm 1 is the case D = 2):
  Step 1  z_d = Prox_{G_eps; eta}(Gamma_d + A_d u_d)                  (eq. updateZ)
          v_{i1,i2} = (pi u_i1 + pi u_i2 + Lam_{i1,i2} + Lam_{i2,i1}) / 2   (eq. updateV-multi)
  Step 2  Gamma_d += A_d u_d - z_d                                     (eq. updateM-1-multi)
  Step 3  u_d = (eta A_d*A_d + r sum_pairs pi^T pi)^{-1}
                (eta A_d*(z_d - Gamma_d) + r sum_pairs pi^T (v - Lam_{d,.}))
          with A_d*A_d = diag(sum_j S_j^T |w|^2) (eq. AtA) and sum pi^T pi = k_d
  Step 4  Lam_{d,d'} += pi_{d,d'} u_d - v_{d,d'}                        (eq. updateM-2-multi;
          the printed v_{i2,i1} in its second line is read as the shared v_{i1,i2})
Initialisation (Step 0): u_d = 1, Gamma = 0, Lam = 0; v^0 and z^0 are never read.
Pixels whose denominator eta*den + r*k vanishes (unilluminated and in no
overlap) keep their value: the sample border of ones of Sec. 4.

Stopping measures (Sec. 4): RF^n = sum_d || |A_d u_d^n| - sqrt(f_d) ||_1 / sum_d ||sqrt(f_d)||_1,
RE^n = max_d ||u_d^n - u_d^{n-1}|| / ||u_d^n||, SNR = -10 log10(||u_r - u_g||^2 / ||u_r||^2).
Merge (Sec. 4): average the subdomain copies where they overlap.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import operators as ops
from .geometry import Geometry, multiplicity, neighbours
from .stagm import G_eps, prox


@dataclass
class OD2PState:
    u: list                      # u_d, complex128 arrays on Omega_d
    gamma: np.ndarray            # Gamma_j, complex128 [J,p,p]
    lam: dict                    # (d, d') -> complex128 array on Omega_d cap Omega_d'
    v: dict = field(default_factory=dict)   # (i1, i2), i1 < i2 -> last consensus value
    z: np.ndarray | None = None  # last z (kept for the Lagrangian / stationarity checks)
    it: int = 0

    def copy(self) -> "OD2PState":
        return OD2PState(u=[a.copy() for a in self.u], gamma=self.gamma.copy(),
                         lam={k: a.copy() for k, a in self.lam.items()},
                         v={k: a.copy() for k, a in self.v.items()},
                         z=None if self.z is None else self.z.copy(), it=self.it)


def init_state(geom: Geometry, u0: complex = 1.0 + 0.0j) -> OD2PState:
    """Step 0: u_d = u0 (1 in the paper), Gamma = 0, Lam = 0."""
    p = geom.p
    u = [np.full(geom.shape(d), u0, dtype=np.complex128) for d in range(geom.D)]
    gamma = np.zeros((geom.J, p, p), dtype=np.complex128)
    lam = {}
    for (i1, i2, rc) in geom.pairs:
        shp = (rc[2] - rc[0], rc[3] - rc[1])
        lam[(i1, i2)] = np.zeros(shp, dtype=np.complex128)
        lam[(i2, i1)] = np.zeros(shp, dtype=np.complex128)
    return OD2PState(u=u, gamma=gamma, lam=lam)


def local_offsets(geom: Geometry, d: int) -> np.ndarray:
    js = geom.frames_of[d]
    return geom.offsets[js] - geom.rects[d, :2][None, :]


def subdomain_illumination(geom: Geometry, w: np.ndarray, d: int) -> np.ndarray:
    """den_d = diag(A_d* A_d) on Omega_d."""
    return ops.illumination(w, local_offsets(geom, d), geom.shape(d))


def forward_sub(geom: Geometry, w: np.ndarray, u: list) -> np.ndarray:
    """Stack of A_d u_d over all frames, indexed by global frame id."""
    p = geom.p
    X = np.empty((geom.J, p, p), dtype=np.complex128)
    for d in range(geom.D):
        js = geom.frames_of[d]
        X[js] = ops.forward(u[d], w, local_offsets(geom, d))
    return X


def adjoint_sub(geom: Geometry, w: np.ndarray, frames: np.ndarray, d: int) -> np.ndarray:
    js = geom.frames_of[d]
    return ops.adjoint(frames[js], w, local_offsets(geom, d), geom.shape(d))


def od2pm_step(geom: Geometry, w: np.ndarray, f: np.ndarray, st: OD2PState,
               eps: float, eta: float, r: float, den: list | None = None):
    """One iteration of Algorithm 2.  Returns (new_state, stats).

    ``f`` holds the intensities [J,p,p].  stats = dict(RF=RF(u^n), RE=RE(u^{n+1}),
    G=G_eps(A u^n; f)).
    """
    sf = np.sqrt(f)
    # Step 1 (consensus): v^{n+1} from u^n and Lam^n
    v = {}
    for (i1, i2, rc) in geom.pairs:
        v[(i1, i2)] = 0.5 * (st.u[i1][geom.restrict(i1, rc)] + st.u[i2][geom.restrict(i2, rc)]
                             + st.lam[(i1, i2)] + st.lam[(i2, i1)])
    # Step 1 (frames): z^{n+1} = Prox(Gamma^n + A u^n)
    X = forward_sub(geom, w, st.u)
    z = prox(st.gamma + X, f, eps, eta)
    # Step 2: Gamma^{n+1}
    gamma = st.gamma + X - z
    # Step 3: u^{n+1}
    u_new = []
    for d in range(geom.D):
        num = adjoint_sub(geom, w, z - gamma, d)
        dd = subdomain_illumination(geom, w, d) if den is None else den[d]
        k = multiplicity(geom, d)
        cons = np.zeros(geom.shape(d), dtype=np.complex128)
        for (e, rc) in neighbours(geom, d):
            key = (min(d, e), max(d, e))
            cons[geom.restrict(d, rc)] += v[key] - st.lam[(d, e)]
        denom = eta * dd + r * k
        held = denom == 0
        safe = np.where(held, 1.0, denom)
        u_new.append(np.where(held, st.u[d], (eta * num + r * cons) / safe))
    # Step 4: Lam^{n+1}
    lam = {}
    for (i1, i2, rc) in geom.pairs:
        lam[(i1, i2)] = st.lam[(i1, i2)] + u_new[i1][geom.restrict(i1, rc)] - v[(i1, i2)]
        lam[(i2, i1)] = st.lam[(i2, i1)] + u_new[i2][geom.restrict(i2, rc)] - v[(i1, i2)]
    new = OD2PState(u=u_new, gamma=gamma, lam=lam, v=v, z=z, it=st.it + 1)
    stats = dict(RF=r_factor(X, sf), RE=relative_change(st.u, u_new), G=G_eps(X, f, eps))
    return new, stats


def od2pm_run(geom, w, f, eps, eta, r, n_iter, state=None):
    """n_iter iterations of Algorithm 2 from ``state`` (Step 0 if None)."""
    st = init_state(geom) if state is None else state
    den = [subdomain_illumination(geom, w, d) for d in range(geom.D)]
    hist = []
    for _ in range(n_iter):
        st, s = od2pm_step(geom, w, f, st, eps, eta, r, den=den)
        st.z = None     # only the single-step API keeps z
        hist.append(s)
    return st, hist


def run_until(step, st, measure: str | None, tol: float, max_iter: int):
    """Step 5 of Algorithms 2 and 3 with the stopping rules of Sec. 4.

    ``step(st) -> (st, stats)`` is one iteration; after each one the rule is checked on
    the measures that iteration produced: ``stats["RF"]`` (of the iterate entering it, the
    noise-free rule RF <= 1e-5) or ``stats["RE"]`` (of the iterate it returns, the noisy
    rule RE <= 1e-3); the run also ends after ``max_iter`` iterations.  The output is the
    last iterate.  Returns (state, per-iteration stats); len(stats) iterations ran.
    """
    hist = []
    while len(hist) < max_iter:
        st, s = step(st)
        hist.append(s)
        if measure is not None and s[measure] <= tol:
            break
    return st, hist


def admm_undecomposed(shape, w, offsets, f, eps, eta, n_iter, u0=None, gamma0=None):
    """ADMM without domain decomposition (the D = 1 row of Table 1), written separately.

    z = Prox(Gamma + A u); Gamma += A u - z; u = A*(z - Gamma) / diag(A*A), holding
    unilluminated pixels.  Returns (u, Gamma).
    """
    u = np.ones(shape, dtype=np.complex128) if u0 is None else np.array(u0, dtype=np.complex128)
    p = w.shape[0]
    gamma = np.zeros((len(offsets), p, p), dtype=np.complex128) if gamma0 is None else gamma0.copy()
    den = ops.illumination(w, offsets, shape)
    for _ in range(n_iter):
        X = ops.forward(u, w, offsets)
        y = gamma + X
        z = prox(y, f, eps, eta)
        gamma = y - z
        num = ops.adjoint(z - gamma, w, offsets, shape)
        u = np.where(den > 0, num / np.where(den > 0, den, 1.0), u)
    return u, gamma


# ---------------------------------------------------------------------------
# measures and merge
# ---------------------------------------------------------------------------

def r_factor(X: np.ndarray, sqrt_f: np.ndarray) -> float:
    """RF = || |X| - sqrt(f) ||_1 / || sqrt(f) ||_1 (Sec. 4)."""
    return float(np.sum(np.abs(np.abs(X) - sqrt_f)) / np.sum(sqrt_f))


def relative_change(u_old: list, u_new: list) -> float:
    """RE = max_d ||u_d^n - u_d^{n-1}|| / ||u_d^n|| (Sec. 4)."""
    return float(max(np.linalg.norm(b - a) / np.linalg.norm(b) for a, b in zip(u_old, u_new)))


def merge(geom: Geometry, u: list, fill: complex = 1.0 + 0.0j) -> np.ndarray:
    """Whole image: non-overlap pixels kept, overlaps averaged (Sec. 4); uncovered pixels = fill."""
    acc = np.zeros((geom.h, geom.w), dtype=np.complex128)
    cnt = np.zeros((geom.h, geom.w), dtype=np.int64)
    for d in range(geom.D):
        r0, c0, r1, c1 = geom.rects[d]
        acc[r0:r1, c0:c1] += u[d]
        cnt[r0:r1, c0:c1] += 1
    return np.where(cnt > 0, acc / np.maximum(cnt, 1), fill)


def align_phase(u_r: np.ndarray, u_g: np.ndarray) -> np.ndarray:
    """u_r times the global phase factor that best matches u_g."""
    c = np.vdot(u_r, u_g)
    return u_r * (c / abs(c)) if abs(c) > 0 else u_r


def snr_db(u_r: np.ndarray, u_g: np.ndarray) -> float:
    """SNR(u_r, u_g) = -10 log10(||u_r - u_g||^2 / ||u_r||^2) after global-phase alignment."""
    ua = align_phase(u_r, u_g)
    return float(-10.0 * np.log10(np.linalg.norm(ua - u_g) ** 2 / np.linalg.norm(ua) ** 2))


def augmented_lagrangian(geom, w, f, st: OD2PState, eps, eta, r) -> float:
    """L_m(u, v, z, Lam, Gamma) of eq. augLag-multi-Domain at the stored iterate."""
    X = forward_sub(geom, w, st.u)
    val = G_eps(st.z, f, eps)
    for (i1, i2, rc) in geom.pairs:
        v = st.v[(i1, i2)]
        for a in (i1, i2):
            b = i2 if a == i1 else i1
            res = st.u[a][geom.restrict(a, rc)] - v
            val += r * float(np.real(np.vdot(st.lam[(a, b)], res))) + 0.5 * r * float(np.vdot(res, res).real)
    res = X - st.z
    val += eta * float(np.real(np.vdot(st.gamma, res))) + 0.5 * eta * float(np.vdot(res, res).real)
    return val

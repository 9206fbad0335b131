"""OD2BP (Algorithm 3 of the paper, Sec. 3.2): blind recovery with probe copies per subdomain.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Variables: u_d (image copies), w (shared probe), w_d (probe copies), Delta_d (their
multipliers), Gamma_j, v, Lam.  One iteration, in the order of Algorithm 3:
  Step 1  w^{n+1} = P_O( mean_d (w_d^n + Delta_d^n) )      (eq. blind_w; 1/2 for D=2, 1/D here)
          v^{n+1} as in the non-blind case                 (eq. blind_v)
          Z_j = Prox(Gamma_j + F(w_d^n o S_j u_d^n))       (eq. blind_Z)
  Step 2  Gamma_j += F(w_d^n o S_j u_d^n) - Z_j            (eq. admm_Gamma)
  Step 3  w_d^{n+1} = (eta D_U*(Z - Gamma) + mu (w^{n+1} - Delta_d^n)) / (eta sum_j |S_j u_d^n|^2 + mu)
          with D_U* y = sum_{j in d} conj(S_j u_d^n) o F^{-1} y_j          (eq. blind_W)
  Step 4  u_d^{n+1} = (eta D_W*(Z - Gamma) + r sum pi^T(v - Lam) + gamma u_d^n)
                      / (eta sum_j S_j^T |w_d^{n+1}|^2 + r k_d + gamma)      (eq. blind_U)
  Step 5  Delta_d += w_d^{n+1} - w^{n+1};  Lam += pi u^{n+1} - v^{n+1}      (eqs. admm_Delta, admm_Lambda)
P_O = F^{-1} M F with M the indicator of the probe's Fourier support (the
printed M is 1 on the zero set, read here as 1 on its complement); no mask means
the identity.  mu = inf freezes the probe (w_d = w - Delta_d).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import operators as ops
from .geometry import Geometry, multiplicity, neighbours
from .od2p import local_offsets, r_factor, relative_change
from .stagm import G_eps, prox


@dataclass
class OD2BPState:
    u: list
    w: np.ndarray
    w_sub: list
    delta: list
    gamma: np.ndarray
    lam: dict
    v: dict
    it: int = 0

    def copy(self):
        return OD2BPState(u=[a.copy() for a in self.u], w=self.w.copy(),
                          w_sub=[a.copy() for a in self.w_sub], delta=[a.copy() for a in self.delta],
                          gamma=self.gamma.copy(), lam={k: a.copy() for k, a in self.lam.items()},
                          v={k: a.copy() for k, a in self.v.items()}, it=self.it)


def init_state(geom: Geometry, w0: np.ndarray) -> OD2BPState:
    """u_d = 1, w = w_d = w0, Gamma = Lam = Delta = 0."""
    p = geom.p
    lam = {}
    for (i1, i2, rc) in geom.pairs:
        shp = (rc[2] - rc[0], rc[3] - rc[1])
        lam[(i1, i2)] = np.zeros(shp, dtype=np.complex128)
        lam[(i2, i1)] = np.zeros(shp, dtype=np.complex128)
    return OD2BPState(u=[np.ones(geom.shape(d), dtype=np.complex128) for d in range(geom.D)],
                      w=np.array(w0, dtype=np.complex128),
                      w_sub=[np.array(w0, dtype=np.complex128) for _ in range(geom.D)],
                      delta=[np.zeros((p, p), dtype=np.complex128) for _ in range(geom.D)],
                      gamma=np.zeros((geom.J, p, p), dtype=np.complex128), lam=lam, v={})


def initial_probe(sqrt_f: np.ndarray) -> np.ndarray:
    """The initial probe of the blind tests (Sec. 4, extended tests, following the
    reference it cites there): w0 = (1/J) sum_j F*(sqrt f_j), the mean over the frames
    of the adjoint (inverse, F being unitary) transform of the amplitudes.
    sqrt_f: [J][p][p] in natural frequency order."""
    sf = np.asarray(sqrt_f, dtype=np.float64)
    return np.mean(ops.ifft2(sf.astype(np.complex128)), axis=0)


def project_support(x: np.ndarray, mask) -> np.ndarray:
    """P_O x = F^{-1}(M o F x); mask None is the identity."""
    if mask is None:
        return x.copy()
    return ops.ifft2(np.asarray(mask, dtype=np.float64) * ops.fft2(x))


def od2bp_step(geom: Geometry, f: np.ndarray, st: OD2BPState, eps, eta, r, mu, gamma_p=0.0,
               mask=None):
    """One iteration of Algorithm 3.  Returns (new_state, stats)."""
    D, p = geom.D, geom.p
    sf = np.sqrt(f)
    # Step 1
    w_new = project_support(sum(st.w_sub[d] + st.delta[d] for d in range(D)) / D, mask)
    v = {}
    for (i1, i2, rc) in geom.pairs:
        v[(i1, i2)] = 0.5 * (st.u[i1][geom.restrict(i1, rc)] + st.u[i2][geom.restrict(i2, rc)]
                             + st.lam[(i1, i2)] + st.lam[(i2, i1)])
    X = np.empty((geom.J, p, p), dtype=np.complex128)
    for d in range(D):
        X[geom.frames_of[d]] = ops.forward(st.u[d], st.w_sub[d], local_offsets(geom, d))
    z = prox(st.gamma + X, f, eps, eta)
    # Step 2
    gamma = st.gamma + X - z
    t = z - gamma
    phi = ops.ifft2(t)                      # F^{-1}(Z - Gamma), per frame
    # Step 3
    w_sub_new = []
    for d in range(D):
        loc = local_offsets(geom, d)
        js = geom.frames_of[d]
        num_w = np.zeros((p, p), dtype=np.complex128)
        den_w = np.zeros((p, p), dtype=np.float64)
        for jj, off in zip(js, loc):
            patch = ops.gather(st.u[d], off, p)
            num_w += np.conj(patch) * phi[jj]
            den_w += np.abs(patch) ** 2
        if np.isinf(mu):
            w_sub_new.append(w_new - st.delta[d])
        else:
            w_sub_new.append((eta * num_w + mu * (w_new - st.delta[d])) / (eta * den_w + mu))
    # Step 4
    u_new = []
    for d in range(D):
        loc = local_offsets(geom, d)
        js = geom.frames_of[d]
        num = np.zeros(geom.shape(d), dtype=np.complex128)
        den = np.zeros(geom.shape(d), dtype=np.float64)
        for jj, off in zip(js, loc):
            ops.scatter_add(num, np.conj(w_sub_new[d]) * phi[jj], off)
            ops.scatter_add(den, np.abs(w_sub_new[d]) ** 2, off)
        k = multiplicity(geom, d)
        cons = np.zeros(geom.shape(d), dtype=np.complex128)
        for (e, rc) in neighbours(geom, d):
            cons[geom.restrict(d, rc)] += v[(min(d, e), max(d, e))] - st.lam[(d, e)]
        denom = eta * den + r * k + gamma_p
        held = denom == 0
        safe = np.where(held, 1.0, denom)
        u_new.append(np.where(held, st.u[d], (eta * num + r * cons + gamma_p * st.u[d]) / safe))
    # Step 5
    delta = [st.delta[d] + w_sub_new[d] - w_new for d in range(D)]
    lam = {}
    for (i1, i2, rc) in geom.pairs:
        lam[(i1, i2)] = st.lam[(i1, i2)] + u_new[i1][geom.restrict(i1, rc)] - v[(i1, i2)]
        lam[(i2, i1)] = st.lam[(i2, i1)] + u_new[i2][geom.restrict(i2, rc)] - v[(i1, i2)]
    new = OD2BPState(u=u_new, w=w_new, w_sub=w_sub_new, delta=delta, gamma=gamma, lam=lam, v=v,
                     it=st.it + 1)
    stats = dict(RF=r_factor(X, sf), RE=relative_change(st.u, u_new), G=G_eps(X, f, eps))
    return new, stats


def od2bp_run(geom, f, w0, eps, eta, r, mu, n_iter, gamma_p=0.0, mask=None, state=None):
    st = init_state(geom, w0) if state is None else state
    hist = []
    for _ in range(n_iter):
        st, s = od2bp_step(geom, f, st, eps, eta, r, mu, gamma_p, mask)
        hist.append(s)
    return st, hist

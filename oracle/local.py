"""FP64 oracle: one iteration of Algorithm 2 or 3 evaluated on chosen subdomains only.

TEST INFRASTRUCTURE ONLY (see the package docstring).

At the full problem sizes a whole oracle iteration takes too long for a test, but each
output of an iteration reads little of the iterate n: the frames of subdomain d (Steps 1-2)
read only u_d and their own Gamma_j; u_d^{n+1} (Step 3) reads those frames, u_d and, through
the consensus v (Step 1), its neighbours' u and the multipliers of its pairs; its
multipliers Lam_{d,.}^{n+1} (Step 4) read u_d^{n+1} and v.  In the blind case (Alg. 3) the
shared probe reads every copy and multiplier (p x p each) and the copy w_d reads the frames
of d.  These functions take the iterate n as the parts they read and return iterate n+1 on
the chosen subdomains, with the equations of od2pm_step and od2bp_step.
"""
from __future__ import annotations

import numpy as np

from . import operators as ops
from .blind import project_support
from .geometry import multiplicity, neighbours
from .od2p import local_offsets
from .stagm import prox


def _consensus(geom, d, u, lam):
    """v_{d,e} (Step 1, eq. updateV-multi) for every neighbour e, and sum_e (v - Lam_{d,e}) on Omega_d."""
    vs, cons = {}, np.zeros(geom.shape(d), dtype=np.complex128)
    for (e, rc) in neighbours(geom, d):
        v = 0.5 * (u[d][geom.restrict(d, rc)] + u[e][geom.restrict(e, rc)] + lam[(d, e)] + lam[(e, d)])
        vs[e] = v
        cons[geom.restrict(d, rc)] += v - lam[(d, e)]
    return vs, cons


def _frames(geom, d, w, u, gamma, f, eps, eta):
    """Steps 1-2 on the frames of d: (ids, Gamma^{n+1}, Z - Gamma^{n+1})."""
    js = geom.frames_of[d]
    X = ops.forward(u[d], w, local_offsets(geom, d))
    G = np.stack([gamma[j] for j in js])
    z = prox(G + X, np.stack([f[j] for j in js]), eps, eta)
    Gn = G + X - z
    return js, Gn, z - Gn


def od2pm_step_local(geom, w, f, u, lam, gamma, eps, eta, r, subs):
    """Algorithm 2 on the subdomains ``subs``.  u: every u_d^n; lam: every Lam^n;
    gamma, f: indexable by frame id (at least the frames of subs).  Returns
    dict(u={d: u_d^{n+1}}, gamma={j: Gamma_j^{n+1}}, lam={(d, e): Lam_{d,e}^{n+1}})."""
    out = dict(u={}, gamma={}, lam={})
    for d in subs:
        js, Gn, t = _frames(geom, d, w, u, gamma, f, eps, eta)
        out["gamma"].update({j: Gn[k] for k, j in enumerate(js)})
        loc = local_offsets(geom, d)
        num = ops.adjoint(t, w, loc, geom.shape(d))
        den = ops.illumination(w, loc, geom.shape(d))
        vs, cons = _consensus(geom, d, u, lam)
        denom = eta * den + r * multiplicity(geom, d)
        held = denom == 0
        un = np.where(held, u[d], (eta * num + r * cons) / np.where(held, 1.0, denom))
        out["u"][d] = un
        for (e, rc) in neighbours(geom, d):
            out["lam"][(d, e)] = lam[(d, e)] + un[geom.restrict(d, rc)] - vs[e]
    return out


def od2bp_step_local(geom, f, u, lam, gamma, w_sub, delta, eps, eta, r, mu, subs, gamma_p=0.0, mask=None):
    """Algorithm 3 on the subdomains ``subs`` (w_sub, delta: every copy and multiplier).
    Returns the dict of od2pm_step_local plus w (the shared probe w^{n+1}) and
    w_sub, delta ({d: ...})."""
    D, p = geom.D, geom.p
    w_new = project_support(sum(w_sub[d] + delta[d] for d in range(D)) / D, mask)
    out = dict(u={}, gamma={}, lam={}, w=w_new, w_sub={}, delta={})
    for d in subs:
        js, Gn, t = _frames(geom, d, w_sub[d], u, gamma, f, eps, eta)
        out["gamma"].update({j: Gn[k] for k, j in enumerate(js)})
        phi = ops.ifft2(t)
        loc = local_offsets(geom, d)
        # Step 3: the probe copy (eq. blind_W)
        num_w = np.zeros((p, p), dtype=np.complex128)
        den_w = np.zeros((p, p), dtype=np.float64)
        for k, off in enumerate(loc):
            patch = ops.gather(u[d], off, p)
            num_w += np.conj(patch) * phi[k]
            den_w += np.abs(patch) ** 2
        ws = (w_new - delta[d]) if np.isinf(mu) else (eta * num_w + mu * (w_new - delta[d])) / (eta * den_w + mu)
        out["w_sub"][d] = ws
        out["delta"][d] = delta[d] + ws - w_new
        # Step 4: the U-step (eq. blind_U) with the new copy
        num = np.zeros(geom.shape(d), dtype=np.complex128)
        den = np.zeros(geom.shape(d), dtype=np.float64)
        for k, off in enumerate(loc):
            ops.scatter_add(num, np.conj(ws) * phi[k], off)
            ops.scatter_add(den, np.abs(ws) ** 2, off)
        vs, cons = _consensus(geom, d, u, lam)
        denom = eta * den + r * multiplicity(geom, d) + gamma_p
        held = denom == 0
        un = np.where(held, u[d], (eta * num + r * cons + gamma_p * u[d]) / np.where(held, 1.0, denom))
        out["u"][d] = un
        for (e, rc) in neighbours(geom, d):
            out["lam"][(d, e)] = lam[(d, e)] + un[geom.restrict(d, rc)] - vs[e]
    return out

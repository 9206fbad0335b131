"""FP64 oracle: automatic overlap penalty by residual balancing.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper fixes the penalties by hand and names their automatic choice as future work
(Sec. 4.3, Sec. 5).  This follows the residual-balancing rule of He, Yang and Wang
(J. Optim. Theory Appl. 106, 2000) in the form of Boyd et al., "Distributed
Optimization and Statistical Learning via the Alternating Direction Method of
Multipliers" (2011), Sec. 3.4.1, applied to the consensus constraints
pi_{d,d'} u_d = v_{d,d'} of Algorithm 2 with their penalty r:

  primal residual   ||pi u^{n+1} - v^{n+1}||   = ||Lam^{n+1} - Lam^n||     (scaled form)
  dual residual     r ||pi (u^{n+1} - u^n)||
  both over all ordered pairs (d, d') and normalised so the rule is scale-free:
  rp = ||pi u^{n+1} - v^{n+1}|| / ||pi u^{n+1}||,   rd = ||pi (u^{n+1} - u^n)|| / ||Lam^{n+1}||
  (the dual residual over the norm of the unscaled multiplier r Lam: r cancels).

After every ``period``-th iteration while the count is at most ``until``:
r <- tau r if rp > mu rd;  r <- r / tau if rd > mu rp;  otherwise r is kept.  The scaled
multipliers follow, Lam <- Lam r_old / r_new, so that the unscaled ones r Lam do not
change.  Stopping the adaptation after ``until`` iterations keeps the tail a plain ADMM
with a fixed penalty.
"""
from __future__ import annotations

import numpy as np

from .od2p import OD2PState, init_state, od2pm_step, subdomain_illumination


def consensus_residuals(geom, old: OD2PState, new: OD2PState) -> dict:
    """Sums of squares over the ordered pairs: P = ||Lam^{n+1} - Lam^n||^2,
    S = ||pi (u^{n+1} - u^n)||^2, U = ||pi u^{n+1}||^2, L = ||Lam^{n+1}||^2."""
    P = S = U = L = 0.0
    for (i1, i2, rc) in geom.pairs:
        for (a, b) in ((i1, i2), (i2, i1)):
            sl = geom.restrict(a, rc)
            P += float(np.sum(np.abs(new.lam[(a, b)] - old.lam[(a, b)]) ** 2))
            S += float(np.sum(np.abs(new.u[a][sl] - old.u[a][sl]) ** 2))
            U += float(np.sum(np.abs(new.u[a][sl]) ** 2))
            L += float(np.sum(np.abs(new.lam[(a, b)]) ** 2))
    return dict(P=P, S=S, U=U, L=L)


def normalised_residuals(res: dict):
    """(rp, rd), or None when a normaliser vanishes."""
    if not (res["U"] > 0.0 and res["L"] > 0.0):
        return None
    return np.sqrt(res["P"] / res["U"]), np.sqrt(res["S"] / res["L"])


def balance_factor(res: dict, mu: float, tau: float) -> float:
    """The rule's factor on r (tau, 1/tau or 1); 1 when a normaliser vanishes."""
    nr = normalised_residuals(res)
    if nr is None:
        return 1.0
    rp, rd = nr
    if rp > mu * rd:
        return tau
    if rd > mu * rp:
        return 1.0 / tau
    return 1.0


def od2pm_run_balanced(geom, w, f, eps, eta, r, n_iter, mu=10.0, tau=2.0, period=10, until=None,
                       state=None, trace=None):
    """n_iter iterations of Algorithm 2 with r chosen by residual balancing.

    Returns (state, per-iteration stats, r after each iteration); ``trace``, if a list,
    receives (iteration, rp, rd) at every check."""
    st = init_state(geom) if state is None else state
    den = [subdomain_illumination(geom, w, d) for d in range(geom.D)]
    until = n_iter if until is None else until
    hist, r_hist = [], []
    for k in range(1, n_iter + 1):
        new, s = od2pm_step(geom, w, f, st, eps, eta, r, den=den)
        new.z = None
        if k % period == 0 and k <= until:
            res = consensus_residuals(geom, st, new)
            if trace is not None:
                trace.append((k, *(normalised_residuals(res) or (np.nan, np.nan))))
            fac = balance_factor(res, mu, tau)
            if fac != 1.0:
                r *= fac
                new.lam = {key: a / fac for key, a in new.lam.items()}
        st = new
        hist.append(s)
        r_hist.append(r)
    return st, hist, r_hist

"""FP64 oracle: automatic penalties (overlap r and data eta) by residual balancing.

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

The same rule applies to the frame constraints A_j u_d = z_j with their penalty eta and
scaled multipliers Gamma (the proximal step and the u-step both use eta):

  primal residual   ||A u^n - z^{n+1}||        = ||Gamma^{n+1} - Gamma^n||
  dual residual     eta ||A (u^{n+1} - u^n)||
  rp = ||Gamma^{n+1} - Gamma^n|| / ||A u^n||,   rd = ||A (u^{n+1} - u^n)|| / ||Gamma^{n+1}||
  with ||A_d x||^2 = sum over Omega_d of den_d |x|^2 (F unitary, eq. AtA), over all frames.

After every ``period``-th iteration while the count is at most ``until``, for each
penalty q in {r, eta} that is balanced: q <- tau q if rp > mu rd; q <- q / tau if
rd > mu rp; otherwise q is kept.  Its scaled multipliers follow (Lam, or Gamma, times
q_old / q_new), so that the unscaled ones q Lam and eta Gamma do not change.  Both
decisions read the same pair of iterates.  Stopping the adaptation after ``until``
iterations keeps the tail a plain ADMM with fixed penalties.
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


def frame_residuals(geom, old: OD2PState, new: OD2PState, den: list) -> dict:
    """Sums of squares for the frame constraints: P = ||Gamma^{n+1} - Gamma^n||^2,
    S = ||A (u^{n+1} - u^n)||^2, U = ||A u^n||^2, L = ||Gamma^{n+1}||^2 (den: den_d)."""
    P = float(np.sum(np.abs(new.gamma - old.gamma) ** 2))
    L = float(np.sum(np.abs(new.gamma) ** 2))
    S = sum(float(np.sum(den[d] * np.abs(new.u[d] - old.u[d]) ** 2)) for d in range(geom.D))
    U = sum(float(np.sum(den[d] * np.abs(old.u[d]) ** 2)) for d in range(geom.D))
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
                       state=None, trace=None, balance_r=True, balance_eta=False, eta_hist=None,
                       trace_eta=None):
    """n_iter iterations of Algorithm 2 with r (and, if asked, eta) chosen by residual
    balancing.

    Returns (state, per-iteration stats, r after each iteration); ``eta_hist``, if a list,
    receives eta after each iteration; ``trace`` and ``trace_eta``, if lists, receive
    (iteration, rp, rd) of the consensus and of the frame constraints at every check."""
    st = init_state(geom) if state is None else state
    den = [subdomain_illumination(geom, w, d) for d in range(geom.D)]
    until = n_iter if until is None else until
    hist, r_hist = [], []
    for k in range(1, n_iter + 1):
        new, s = od2pm_step(geom, w, f, st, eps, eta, r, den=den)
        new.z = None
        if k % period == 0 and k <= until:
            if balance_r:
                res = consensus_residuals(geom, st, new)
                if trace is not None:
                    trace.append((k, *(normalised_residuals(res) or (np.nan, np.nan))))
                fac = balance_factor(res, mu, tau)
                if fac != 1.0:
                    r *= fac
                    new.lam = {key: a / fac for key, a in new.lam.items()}
            if balance_eta:
                res = frame_residuals(geom, st, new, den)
                if trace_eta is not None:
                    trace_eta.append((k, *(normalised_residuals(res) or (np.nan, np.nan))))
                fac = balance_factor(res, mu, tau)
                if fac != 1.0:
                    eta *= fac
                    new.gamma = new.gamma / fac
        st = new
        hist.append(s)
        r_hist.append(r)
        if eta_hist is not None:
            eta_hist.append(eta)
    return st, hist, r_hist

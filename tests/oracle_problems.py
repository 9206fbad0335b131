"""Test helpers: oracle-side problem data built from the seeded synthetic recipes.

Intensities come from the FP64 oracle's forward model, never from the GPU path.
"""
from __future__ import annotations

import numpy as np

import synthetic
from oracle import operators as ops
from oracle.geometry import build_geometry
from oracle.od2p import subdomain_illumination

EPS = 0.5          # truncation used in all of the paper's experiments (Sec. 4)
ETA = 0.1          # data penalty of Sec. 4.1
RHO_R = 0.5        # r = RHO_R * eta * max diag(A*A): scale-free overlap penalty


def oracle_problem(spec, eta=ETA, rho_r=RHO_R, eps=EPS):
    """Draw a spec, synthesise intensities with the oracle forward model and pick penalties."""
    pr = synthetic.draw_problem(spec)
    f0 = ops.intensities(pr["u_true"], pr["w"], pr["offsets"])
    f = synthetic.poisson_counts(f0, spec.peak, pr["rng_poisson"])
    geom = build_geometry(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"])
    den = [subdomain_illumination(geom, pr["w"], d) for d in range(geom.D)]
    dmax = max(float(a.max()) for a in den)
    r = rho_r * eta * dmax
    return dict(pr=pr, f=f, f_clean=f0, geom=geom, den=den, eps=eps, eta=eta, r=r)


def tiny_spec(n=24, p=8, step=4, dy=1, dx=2, jitter=1, seed=11, peak=None, radius=3.0, **kw):
    return synthetic.ProblemSpec(f"tiny{n}_{p}_{step}_{dy}x{dx}", n=n, sigma=2.0, p=p, radius=radius,
                                 quad=0.05, step=step, jitter=jitter, dy=dy, dx=dx, peak=peak,
                                 iters=10, seed=seed, **kw)

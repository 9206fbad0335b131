"""Write the FP64 oracle's c2 reconstruction after 200 OD2Pm iterations, sampled.

Calls only the oracle and the seeded input recipes.  Output: c2_k200_oracle.npz with
  idx      int64 [S]   flat pixel indices of the 512x512 merged image (seeded sample)
  u        complex128 [S] merged image at those pixels
  norm     float64     Frobenius norm of the whole merged image
  rf, re   float64 [K] RF and RE per iteration (Sec. 4)
Inputs: intensities from the oracle's forward model with seeded Poisson noise, the
probe rounded to complex64 and sqrt(f) rounded to float32 (what the GPU reads).
Run: python tests/golden/make_c2_reference.py   (a few minutes, single thread)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthetic  # noqa: E402
from oracle import operators as ops  # noqa: E402
from oracle.geometry import build_geometry  # noqa: E402
from oracle.od2p import merge, od2pm_run, subdomain_illumination  # noqa: E402

K = 200
S = 8192


def main():
    spec = synthetic.CONFIGS["c2"]
    pr = synthetic.draw_problem(spec)
    f = synthetic.poisson_counts(ops.intensities(pr["u_true"], pr["w"], pr["offsets"]), spec.peak,
                                 pr["rng_poisson"])
    f = np.sqrt(f).astype(np.float32).astype(np.float64) ** 2
    w = pr["w"].astype(np.complex64).astype(np.complex128)
    g = build_geometry(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"])
    eps, eta = 0.5, 0.1
    r = 0.5 * eta * max(float(subdomain_illumination(g, w, d).max()) for d in range(g.D))
    st, hist = od2pm_run(g, w, f, eps, eta, r, K)
    u = merge(g, st.u)
    idx = np.sort(np.random.default_rng(2024).choice(u.size, size=S, replace=False))
    np.savez(os.path.join(HERE, "c2_k200_oracle.npz"), idx=idx, u=u.reshape(-1)[idx], norm=np.linalg.norm(u),
             rf=np.array([h["RF"] for h in hist]), re=np.array([h["RE"] for h in hist]), r=r)
    print("RF", hist[0]["RF"], "->", hist[-1]["RF"], "RE", hist[-1]["RE"])


if __name__ == "__main__":
    main()

"""Write the FP64 oracle's blind reconstruction of the 2048 x 2048 / 6561-frame workload
after K = 10 OD2BP iterations (Alg. 3) from the flat-disk start, sampled, with the
oracle's own sensitivity to a rounding-sized change of its input.

Calls only the oracle and the seeded input recipes.  Stores:
  idx        int64 [S]        seeded sample of merged-image pixels (row-major index)
  u10        complex128 [S]   merged image after 10 iterations at idx
  w10        complex128 [p,p] shared probe after 10 iterations
  norm10     float64          Frobenius norm of the whole merged image after 10
  rf         float64 [10]     RF per iteration (Sec. 4)
  sens10, sens10_w
             float64 [2]      relative distance (sample, probe) between this run and the
                              same run from sqrt(f) multiplied by a seeded factor uniform in
                              1 +- 2^-24 (half a float32 ulp), for two seeds
  sens10_w0, sens10_w0_bf16
             float64 [2]      the same (sample, probe) for the start probe w0 multiplied by
                              a seeded complex factor 1 + d, |Re d|, |Im d| <= 2^-24 (float32)
                              or 2^-17 (a split-BF16 hi + lo pair): at Step 0 y = F(w0 o S_j 1)
                              has near-zeros (the flat disk's Airy rings) whose phase, and so
                              the first Gamma there, is a tie at the transform's resolution
  r, mu      float64          the penalties (r = 0.5 eta max_d den_d(w0), mu = 0.5 eta max_d J_d)
Inputs: the true probe rounded to complex64 for the forward model, sqrt(f) of the seeded
Poisson counts (peak 1e4) rounded to float32, the start w0 = flat disk of radius 40 scaled
to the mean frame energy, rounded to complex64.  eps = 0.5, eta = 0.1.
Run: python tests/golden/make_c5_reference.py   (about 35 minutes, one thread)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthetic  # noqa: E402
from oracle import blind, operators as ops  # noqa: E402
from oracle.geometry import build_geometry  # noqa: E402
from oracle.od2p import merge, subdomain_illumination  # noqa: E402

K = 10
S = 8192
EPS, ETA = 0.5, 0.1
SEEDS = (7, 8)


def inputs():
    spec = synthetic.CONFIGS["c5"]
    pr = synthetic.draw_problem(spec)
    w_true = pr["w"].astype(np.complex64).astype(np.complex128)
    f0 = ops.intensities(pr["u_true"], w_true, pr["offsets"])
    f = synthetic.poisson_counts(f0, spec.peak, pr["rng_poisson"])
    del f0
    sf = np.sqrt(f).astype(np.float32).astype(np.float64)
    w0 = (synthetic.make_probe(spec.p, spec.init_radius, 0.0) * synthetic.problems.blind_init_amplitude(
        float(np.mean(np.sum(sf ** 2, axis=(1, 2)))), spec.init_radius)).astype(np.complex64).astype(np.complex128)
    return spec, pr, sf, w0


def main():
    spec, pr, sf, w0 = inputs()
    g = build_geometry(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"])
    r = 0.5 * ETA * max(float(subdomain_illumination(g, w0, d).max()) for d in range(g.D))
    mu = 0.5 * ETA * max(len(fr) for fr in g.frames_of)
    idx = np.sort(np.random.default_rng(2025).choice(spec.n * spec.n, size=S, replace=False))
    st, hist = blind.od2bp_run(g, sf ** 2, w0, EPS, ETA, r, mu, K)
    u = merge(g, st.u)
    res = dict(idx=idx, u10=u.reshape(-1)[idx], w10=st.w, norm10=np.linalg.norm(u),
               rf=np.array([h["RF"] for h in hist]), r=r, mu=mu)
    print("RF", res["rf"][0], "->", res["rf"][-1], flush=True)
    del st
    sens, sens_w = [], []
    for seed in SEEDS:
        unit = np.random.default_rng(seed).uniform(-1.0, 1.0, sf.shape)
        stp, _ = blind.od2bp_run(g, (sf * (1.0 + 2.0 ** -24 * unit)) ** 2, w0, EPS, ETA, r, mu, K)
        a, b = res["u10"], merge(g, stp.u).reshape(-1)[idx]
        sens.append(np.linalg.norm(a - b) / np.linalg.norm(a))
        sens_w.append(np.linalg.norm(stp.w - res["w10"]) / np.linalg.norm(res["w10"]))
        print("seed", seed, "sens", sens[-1], "sens_w", sens_w[-1], flush=True)
        del stp, unit
    res["sens10"] = np.array(sens)
    res["sens10_w"] = np.array(sens_w)
    for tag, scale in (("", 2.0 ** -24), ("_bf16", 2.0 ** -17)):
        rng = np.random.default_rng(9)
        d = scale * (rng.uniform(-1.0, 1.0, w0.shape) + 1j * rng.uniform(-1.0, 1.0, w0.shape))
        stp, _ = blind.od2bp_run(g, sf ** 2, w0 * (1.0 + d), EPS, ETA, r, mu, K)
        a, b = res["u10"], merge(g, stp.u).reshape(-1)[idx]
        res[f"sens10_w0{tag}"] = np.array([np.linalg.norm(a - b) / np.linalg.norm(a),
                                           np.linalg.norm(stp.w - res["w10"]) / np.linalg.norm(res["w10"])])
        print("w0 perturbation", scale, res[f"sens10_w0{tag}"], flush=True)
        del stp
    np.savez_compressed(os.path.join(HERE, "c5_k10_oracle.npz"), **res)


if __name__ == "__main__":
    main()

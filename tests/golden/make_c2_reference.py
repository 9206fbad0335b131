"""Write the FP64 oracle's c2 reconstructions after K iterations, sampled, together with
the oracle's own sensitivity to a rounding-sized change of its input.

Calls only the oracle and the seeded input recipes.  For each data case (Poisson
counts at peak 1e4 as in the c2 recipe, and the noise-free intensities) it stores,
under the prefix "<case>_":
  u50, u200   complex128 [S] merged image after 50 and 200 OD2Pm iterations at the
              seeded pixel sample idx (int64 [S], shared by the cases)
  norm200     float64     Frobenius norm of the whole merged image after 200
  rf          float64 [K] RF per iteration (Sec. 4)
  err_true    float64     || align(u200) - u_true || / || u_true || on the whole image
  sens50, sens200
              float64     relative distance, on the sample, between this run and
                          the same run from sqrt(f) multiplied by a seeded factor
                          uniform in 1 +- 2^-24 (half a float32 ulp)
  sens50_bf16, sens200_bf16
              float64     the same with 1 +- 2^-17 (the resolution of a split-BF16
                          hi + lo pair)
and r (the overlap penalty, shared).
Inputs: the probe rounded to complex64 and sqrt(f) rounded to float32 (what the GPU
reads).  eps = 0.5, eta = 0.1, r = 0.5 eta max_d den_d.
Run: python tests/golden/make_c2_reference.py   (about 45 minutes, four threads)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthetic  # noqa: E402
from oracle import operators as ops  # noqa: E402
from oracle.geometry import build_geometry  # noqa: E402
from oracle.od2p import align_phase, merge, od2pm_run, subdomain_illumination  # noqa: E402

K = (50, 200)
S = 8192
EPS, ETA = 0.5, 0.1


def snapshots(g, w, sf, r, idx):
    st, done, out, rf = None, 0, {}, []
    for k in K:
        st, hist = od2pm_run(g, w, sf ** 2, EPS, ETA, r, k - done, state=st)
        rf += [h["RF"] for h in hist]
        done = k
        u = merge(g, st.u)
        out[k] = u
    return out, np.array(rf)


def main():
    spec = synthetic.CONFIGS["c2"]
    pr = synthetic.draw_problem(spec)
    w = pr["w"].astype(np.complex64).astype(np.complex128)
    g = build_geometry(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"])
    r = 0.5 * ETA * max(float(subdomain_illumination(g, w, d).max()) for d in range(g.D))
    idx = np.sort(np.random.default_rng(2024).choice(spec.n * spec.n, size=S, replace=False))
    f0 = ops.intensities(pr["u_true"], pr["w"], pr["offsets"])
    cases = {"poisson": synthetic.poisson_counts(f0, spec.peak, pr["rng_poisson"]), "clean": f0}
    res = dict(idx=idx, r=r)
    for name, f in cases.items():
        sf = np.sqrt(f).astype(np.float32).astype(np.float64)
        snap, rf = snapshots(g, w, sf, r, idx)
        unit = np.random.default_rng(7).uniform(-1.0, 1.0, sf.shape)
        for tag, scale in (("", 2.0 ** -24), ("_bf16", 2.0 ** -17)):
            snap_p, _ = snapshots(g, w, sf * (1.0 + scale * unit), r, idx)
            for k in K:
                a, b = snap[k].reshape(-1)[idx], snap_p[k].reshape(-1)[idx]
                res[f"{name}_u{k}"] = a
                res[f"{name}_sens{k}{tag}"] = np.linalg.norm(a - b) / np.linalg.norm(a)
        u = snap[K[-1]]
        res[f"{name}_norm200"] = np.linalg.norm(u)
        res[f"{name}_rf"] = rf
        res[f"{name}_err_true"] = np.linalg.norm(align_phase(u, pr["u_true"]) - pr["u_true"]) / np.linalg.norm(
            pr["u_true"])
        print(name, "RF", rf[0], "->", rf[-1], "err_true", res[f"{name}_err_true"],
              "sens", res[f"{name}_sens50"], res[f"{name}_sens200"],
              "sens_bf16", res[f"{name}_sens50_bf16"], res[f"{name}_sens200_bf16"], flush=True)
    np.savez(os.path.join(HERE, "c2_k200_oracle.npz"), **res)


if __name__ == "__main__":
    main()

"""GPU parity of OD2BP (Algorithm 3): frame sweep with probe copies, probe update
(w, w_d, Delta) and the U-step, against the FP64 oracle."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import synthetic
from oracle import blind
from tests.gpu_util import dev_c64, gpu_plan, host, rel, rel_list, rounded_inputs
from tests.oracle_problems import oracle_problem, tiny_spec

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)


def _blind_setup(spec, mu_scale=0.5, gamma=0.0, mask=None):
    P = oracle_problem(spec)
    w_true, _, f = rounded_inputs(P)
    p = spec.p
    w0 = synthetic.make_probe(p, spec.radius * 0.85, 0.0)
    w0 = (w0 * np.sqrt(f.sum(axis=(1, 2)).mean() / max(np.sum(np.abs(w0) ** 2), 1e-30)))
    w0 = w0.astype(np.complex64).astype(np.complex128)
    g = P["geom"]
    mu = mu_scale * P["eta"] * max(len(fr) for fr in g.frames_of)
    plan = gpu_plan(P, blind=True, mu=mu, gamma=gamma, mask=mask)
    st = plan.new_state(w0=dev_c64(w0))
    return P, f, g, w0, mu, plan, st


def _compare(st, ost, tol):
    e_u = rel_list([host(t) for t in st.u_sub()], ost.u)
    e_w = rel(host(st.probe()), ost.w)
    e_ws = rel(host(st.probe_copies()), np.stack(ost.w_sub))
    e_g = rel(host(st.gamma()), ost.gamma)
    dl = np.stack(ost.delta)
    e_d = rel(host(st.probe_multipliers()), dl) / 50 if np.linalg.norm(dl) > 0 else 0.0  # small differences
    errs = dict(u=e_u, w=e_w, w_sub=e_ws, gamma=e_g, delta_over_50=e_d)
    assert max(errs.values()) <= tol, errs


@pytest.mark.parametrize("gamma", [0.0, 0.3])
def test_blind_iterations_parity(gamma):
    spec = tiny_spec(n=128, p=32, step=8, jitter=1, dy=2, dx=2, radius=12, peak=1e4)
    say("blind parity gamma", gamma)
    P, f, g, w0, mu, plan, st = _blind_setup(spec, gamma=gamma)
    stats = host(plan.iterate(st, 1, stats=True))
    ost, hist = blind.od2bp_run(g, f, w0, P["eps"], P["eta"], P["r"], mu, 1, gamma_p=gamma)
    _compare(st, ost, 1e-5)
    assert abs(stats[0, 0] - hist[0]["RF"]) <= 1e-5 * hist[0]["RF"]
    plan.iterate(st, 9)
    ost, _ = blind.od2bp_run(g, f, w0, P["eps"], P["eta"], P["r"], mu, 9, gamma_p=gamma, state=ost)
    _compare(st, ost, 1e-3)   # K-iteration reconstruction bound


def test_blind_with_support_mask():
    spec = tiny_spec(n=128, p=32, step=8, jitter=0, dy=1, dx=2, radius=12, peak=None)
    say("blind with support mask")
    k = np.fft.fftfreq(32) * 32
    mask = ((k[:, None] ** 2 + k[None, :] ** 2) <= 10 ** 2).astype(np.uint8)
    P, f, g, w0, mu, plan, st = _blind_setup(spec, mask=mask)
    plan.iterate(st, 1)
    ost, _ = blind.od2bp_run(g, f, w0, P["eps"], P["eta"], P["r"], mu, 1, mask=mask)
    _compare(st, ost, 1e-5)
    plan.iterate(st, 2)
    ost, _ = blind.od2bp_run(g, f, w0, P["eps"], P["eta"], P["r"], mu, 2, mask=mask, state=ost)
    _compare(st, ost, 1e-3)   # K-iteration reconstruction bound
    # the shared probe's spectrum vanishes off the support
    spec_w = np.fft.fft2(host(st.probe()), norm="ortho")
    assert np.abs(spec_w[mask == 0]).max() <= 1e-5 * np.abs(spec_w).max()


def test_blind_p64_single_run():
    spec = tiny_spec(n=192, p=64, step=16, jitter=2, dy=2, dx=2, radius=24, peak=1e4)
    say("blind p64")
    P, f, g, w0, mu, plan, st = _blind_setup(spec)
    plan.iterate(st, 5)
    ost, _ = blind.od2bp_run(g, f, w0, P["eps"], P["eta"], P["r"], mu, 5)
    _compare(st, ost, 1e-3)   # K-iteration reconstruction bound


def test_blind_p128_parity():
    """p = 128 (the blind workload's probe size).  The U-step divides by the probe copy's
    illumination; with a disk probe the frame corners light some pixels at 1e-6 of the
    maximum, where the division amplifies rounding differences without bound, so u is
    compared on the pixels lit at >= 1e-3 of the maximum (all of them in the p = 32
    test above).  Gamma = y - Prox(y) is a difference of nearly equal spectra at p = 128
    (relative cancellation of about 1e-4 in FP32), so it gets the K-iteration bound."""
    from oracle.od2p import subdomain_illumination
    spec = tiny_spec(n=256, p=128, step=16, jitter=2, dy=2, dx=2, radius=48, peak=1e4)
    say("blind p128")
    P, f, g, w0, mu, plan, st = _blind_setup(spec)
    lit = [subdomain_illumination(g, w0, d) for d in range(g.D)]
    lit = [a >= 1e-3 * a.max() for a in lit]

    def check(ost, tol_u):
        got = [host(t) for t in st.u_sub()]
        num = sum(np.sum(np.abs(got[d][lit[d]] - ost.u[d][lit[d]]) ** 2) for d in range(g.D))
        den = sum(np.sum(np.abs(ost.u[d][lit[d]]) ** 2) for d in range(g.D))
        errs = dict(u_lit=float(np.sqrt(num / den)), w=rel(host(st.probe()), ost.w),
                    w_sub=rel(host(st.probe_copies()), np.stack(ost.w_sub)), gamma=rel(host(st.gamma()), ost.gamma))
        say("blind p128 errors", errs)
        assert errs["u_lit"] <= tol_u, errs
        assert max(errs["w"], errs["w_sub"], errs["gamma"]) <= 1e-3, errs

    stats = host(plan.iterate(st, 1, stats=True))
    ost, hist = blind.od2bp_run(g, f, w0, P["eps"], P["eta"], P["r"], mu, 1)
    check(ost, 1e-4)
    assert abs(stats[0, 0] - hist[0]["RF"]) <= 1e-5 * hist[0]["RF"]
    plan.iterate(st, 4)
    ost, _ = blind.od2bp_run(g, f, w0, P["eps"], P["eta"], P["r"], mu, 4, state=ost)
    check(ost, 1e-3)   # K-iteration reconstruction bound


@pytest.mark.parametrize("n,p,step,rad", [(128, 32, 8, 12), (192, 64, 16, 24), (256, 128, 32, 48)], ids=["p32", "p64", "p128"])
def test_initial_probe_matches_oracle(n, p, step, rad):
    """w0 = (1/J) sum_j F*(sqrt f_j) (Sec. 4, extended tests) from the bound amplitudes."""
    from tests.gpu_util import gpu_plan
    from tests.oracle_problems import oracle_problem
    spec = tiny_spec(n=n, p=p, step=step, jitter=2, dy=2, dx=2, radius=rad, peak=1e4)
    say("initial probe", p)
    P = oracle_problem(spec)
    _, sf32, _ = rounded_inputs(P)
    plan = gpu_plan(P, blind=True, mu=1.0)
    got = host(plan.blind_initial_probe())
    want = blind.initial_probe(sf32.astype(np.float64))
    assert rel(got, want) <= 1e-5, rel(got, want)


def test_initial_probe_per_problem_of_a_batch():
    from tests.gpu_util import dev_f32
    import paper_2011_00162_amd as odp
    from tests.oracle_problems import oracle_problem
    specs = [tiny_spec(n=128, p=32, step=8, jitter=1, dy=1, dx=2, radius=12, peak=1e4),
             tiny_spec(n=160, p=32, step=8, jitter=2, dy=2, dx=2, radius=12, peak=1e3)]
    Ps = [oracle_problem(s) for s in specs]
    sfs = [rounded_inputs(P)[1] for P in Ps]
    probs = [dict(H=s.n, W=s.n, p=s.p, offsets=P["pr"]["offsets"], frame_sub=P["pr"]["frame_sub"], r=1.0)
             for s, P in zip(specs, Ps)]
    plan = odp.Plan.batch(probs)
    w = torch.stack([dev_c64(np.asarray(P["pr"]["w"])) for P in Ps])
    plan.bind(dev_f32(np.concatenate(sfs)), w)
    got = host(plan.blind_initial_probe())
    for i, sf in enumerate(sfs):
        assert rel(got[i], blind.initial_probe(sf.astype(np.float64))) <= 1e-5, i

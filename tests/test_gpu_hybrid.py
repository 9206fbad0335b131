"""GPU parity of the hybrid frame transform (ODP_HYBRID_MFMA: the radix-16 stages of the
FFT as split-BF16 products on the matrix cores, the radix-4/8 stage in FP32) against the
FP64 oracle, p = 64 and 128.

Each split-BF16 stage is exact to about 2^-16 per product (hi*hi + hi*lo + lo*hi of the
bf16 splits); a frame passes through four of them per iteration (two per transform), so
one iteration is held to 1e-4 (the split-BF16 bound of the DFT path), in norm and element
by element (tests.gpu_util), and reconstructions after K iterations to 1e-3.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import synthetic
import paper_2011_00162_amd as odp
from oracle import operators as ops
from oracle.od2p import init_state, merge, od2pm_run, od2pm_step
from tests.gpu_util import (dev_c64, dev_f32, gamma_elem_err, host, lam_elem_err, oracle_to_state, rel, rel_list,
                            rounded_inputs, state_to_oracle, u_elem_err, u_weights)
from tests.oracle_problems import oracle_problem, tiny_spec

pytestmark = pytest.mark.gpu

TOL1 = 1e-4     # one iteration, split BF16


def say(*a):
    print("[gpu]", *a, flush=True)


def _plan(P, transform=odp.ODP_HYBRID_MFMA, **kw):
    spec = P["pr"]["spec"]
    w, sf32, _ = rounded_inputs(P)
    plan = odp.Plan(spec.n, spec.n, spec.p, P["pr"]["offsets"], P["pr"]["frame_sub"], eps=P["eps"],
                    eta=kw.get("eta", P["eta"]), r=P["r"], transform=transform, blind=kw.get("blind", False),
                    mu=kw.get("mu", 0.0))
    plan.bind(dev_f32(sf32), dev_c64(w))
    return plan


def _random_state(g, seed):
    rng = np.random.default_rng(seed)
    r64 = lambda x: x.astype(np.complex64).astype(np.complex128)
    ost = init_state(g)
    ost.u = [r64(1 + 0.3 * (rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape))) for a in ost.u]
    ost.gamma = r64(0.05 * (rng.standard_normal(ost.gamma.shape) + 1j * rng.standard_normal(ost.gamma.shape)))
    ost.lam = {k: r64(0.1 * (rng.standard_normal(v.shape) + 1j * rng.standard_normal(v.shape)))
               for k, v in ost.lam.items()}
    return ost


CASES = [
    ("p64_eta0.1", tiny_spec(n=256, p=64, step=16, jitter=2, dy=2, dx=3, radius=24, peak=1e3), 0.1),
    ("p64_eta2", tiny_spec(n=256, p=64, step=16, jitter=2, dy=2, dx=3, radius=24, peak=1e3), 2.0),
    ("p128", tiny_spec(n=320, p=128, step=32, jitter=2, dy=2, dx=2, radius=48, peak=1e3), 0.1),
]


@pytest.mark.parametrize("name,spec,eta", CASES, ids=[c[0] for c in CASES])
def test_hybrid_one_iteration_from_random_state(name, spec, eta):
    say("hybrid one iteration", name)
    P = oracle_problem(spec, eta=eta)
    g = P["geom"]
    w, _, f = rounded_inputs(P)
    plan = _plan(P, eta=eta)
    st = plan.new_state()
    ost = _random_state(g, 7)
    oracle_to_state(ost, st)
    stats = host(plan.iterate(st, 1, stats=True))
    new, ostats = od2pm_step(g, w, f, ost, P["eps"], eta, P["r"])
    got = state_to_oracle(st)
    e = dict(u=rel_list(got.u, new.u), gamma=rel(got.gamma, new.gamma),
             lam=max(rel(got.lam[k], new.lam[k]) for k in new.lam),
             RF=abs(stats[0, 0] - ostats["RF"]) / ostats["RF"])
    el = dict(u_elem=u_elem_err(got.u, new.u, u_weights(g, lambda d: w, eta, P["r"]), floor="rms"),
              gamma_elem=gamma_elem_err(got.gamma, new.gamma, new.gamma + new.z, np.sqrt(f), P["eps"], eta),
              lam_elem=lam_elem_err(got.lam, new.lam, new.u, g))
    say("hybrid, one iteration vs FP64:", {k: f"{v:.2e}" for k, v in {**e, **el}.items()})
    assert max(e.values()) <= TOL1, e
    assert max(el.values()) <= TOL1, el


@pytest.mark.parametrize("p", [64, 128])
def test_hybrid_forward_transform_matches_fft_sweep(p):
    """Gamma after one sweep from Gamma = 0 and a known u: the hybrid and the FP32 FFT sweep
    against the oracle's y - Prox(y) on the same frames, frame by frame."""
    n, step = (192, 16) if p == 64 else (320, 32)
    spec = tiny_spec(n=n, p=p, step=step, jitter=1, dy=1, dx=2, radius=0.38 * p, peak=None)
    say("hybrid transform frames", p)
    P = oracle_problem(spec)
    g = P["geom"]
    w, _, f = rounded_inputs(P)
    ost = _random_state(g, 11)
    ost.gamma[:] = 0
    new, _ = od2pm_step(g, w, f, ost, P["eps"], P["eta"], P["r"])
    for tr in (odp.ODP_FFT_F32, odp.ODP_HYBRID_MFMA):
        plan = _plan(P, transform=tr)
        st = plan.new_state()
        oracle_to_state(ost, st)
        plan.frame_sweep(st)
        torch.cuda.synchronize()
        G = host(st.gamma())
        per_frame = (np.linalg.norm((G - new.gamma).reshape(g.J, -1), axis=1)
                     / np.linalg.norm(new.gamma.reshape(g.J, -1), axis=1))
        say("transform", tr, "worst frame rel error of Gamma", f"{per_frame.max():.2e}")
        assert per_frame.max() <= (1e-5 if tr == odp.ODP_FFT_F32 else TOL1)


@pytest.mark.parametrize("p,K", [(64, 50), (128, 10)])
def test_hybrid_reconstruction_within_bound(p, K):
    n, step = (256, 16) if p == 64 else (320, 32)
    spec = tiny_spec(n=n, p=p, step=step, jitter=2, dy=2, dx=2, radius=0.375 * p, peak=None)
    say("hybrid reconstruction", p, K)
    P = oracle_problem(spec)
    g = P["geom"]
    w, _, f = rounded_inputs(P)
    plan = _plan(P)
    st = plan.new_state()
    plan.iterate(st, K)
    ost, _ = od2pm_run(g, w, f, P["eps"], P["eta"], P["r"], K)
    err = rel(host(plan.merge(st)), merge(g, ost.u))
    say(f"hybrid, merged image after {K} iterations, relative error vs FP64: {err:.2e}")
    assert err <= 1e-3


def test_hybrid_c2_full_size_iterations():
    spec = synthetic.CONFIGS["c2"]
    say("hybrid c2 full size, 3 iterations")
    P = oracle_problem(spec)
    g = P["geom"]
    w, _, f = rounded_inputs(P)
    plan = _plan(P)
    st = plan.new_state()
    plan.iterate(st, 3)
    ost, _ = od2pm_run(g, w, f, P["eps"], P["eta"], P["r"], 3)
    got = state_to_oracle(st)
    e = dict(u=rel_list(got.u, ost.u), gamma=rel(got.gamma, ost.gamma))
    say("hybrid, c2 after 3 iterations:", {k: f"{v:.2e}" for k, v in e.items()})
    assert max(e.values()) <= TOL1, e


def test_hybrid_blind_from_advanced_state():
    """Blind (Alg. 3) at p = 128 with the hybrid sweep: one iteration from the oracle's
    third iterate (no Step-0 ties of the flat disk's spectrum)."""
    from oracle import blind
    from tests.gpu_util import u_weighted_rel
    from oracle.od2p import subdomain_illumination
    spec = tiny_spec(n=256, p=128, step=16, jitter=2, dy=2, dx=2, radius=48, peak=1e4)
    say("hybrid blind p128")
    P = oracle_problem(spec)
    _, _, f = rounded_inputs(P)
    g = P["geom"]
    w0 = synthetic.make_probe(128, 48 * 0.85, 0.0)
    w0 = (w0 * np.sqrt(f.sum(axis=(1, 2)).mean() / np.sum(np.abs(w0) ** 2))).astype(np.complex64).astype(np.complex128)
    mu = 0.5 * P["eta"] * max(len(fr) for fr in g.frames_of)
    o3, _ = blind.od2bp_run(g, f, w0, P["eps"], P["eta"], P["r"], mu, 3)
    r64 = lambda x: x.astype(np.complex64).astype(np.complex128)
    o3.u = [r64(a) for a in o3.u]
    o3.gamma = r64(o3.gamma)
    o3.lam = {k: r64(v) for k, v in o3.lam.items()}
    o3.w, o3.w_sub, o3.delta = r64(o3.w), [r64(a) for a in o3.w_sub], [r64(a) for a in o3.delta]
    plan = _plan(P, blind=True, mu=mu)
    st = plan.new_state(w0=dev_c64(w0))
    oracle_to_state(o3, st)
    st.probe().copy_(torch.from_numpy(o3.w.astype(np.complex64)))
    st.probe_copies().copy_(torch.from_numpy(np.stack(o3.w_sub).astype(np.complex64)))
    st.probe_multipliers().copy_(torch.from_numpy(np.stack(o3.delta).astype(np.complex64)))
    plan.iterate(st, 1)
    o4, _ = blind.od2bp_step(g, f, o3, P["eps"], P["eta"], P["r"], mu)
    den = [subdomain_illumination(g, o4.w_sub[d], d) for d in range(g.D)]
    e = dict(u_weighted=u_weighted_rel([host(t) for t in st.u_sub()], o4.u, den),
             gamma=rel(host(st.gamma()), o4.gamma), w_sub=rel(host(st.probe_copies()), np.stack(o4.w_sub)),
             w=rel(host(st.probe()), o4.w))
    say("hybrid blind, one iteration vs FP64:", {k: f"{v:.2e}" for k, v in e.items()})
    assert max(e.values()) <= TOL1, e


def test_hybrid_refused_where_not_built():
    spec = tiny_spec(n=96, p=32, step=8, jitter=1, dy=1, dx=2, radius=12, peak=None)
    P = oracle_problem(spec)
    with pytest.raises(odp.OdpError):
        _plan(P)

"""Parity at the full sizes of the benchmark workloads, in the launch configuration the
benchmark times, on outputs the FP64 oracle computes one subdomain at a time
(oracle.local): one iteration from an advanced state, compared on chosen subdomains
(their u, the Gamma of their frames, their multipliers and, blind, their probe copies).

* 2048 x 2048 image, 6561 frames of 128 x 128, 8 x 8 subdomains, Poisson peak 1e4:
  known probe, and blind from the flat-disk start (plan.iterate, as the benchmark);
* the 64-problem batch (two batch plans by probe size, autotuned, one graph): one
  problem of each probe size.
The amplitude loss at its full size (1024 x 1024, 841 frames of 128 x 128) is compared
on every output in test_gpu_loss.py."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import synthetic
import paper_2011_00162_amd as odp
from oracle import local, operators as ops
from oracle.geometry import build_geometry
from oracle.od2p import subdomain_illumination
from tests.gpu_util import dev_c64, dev_f32, host, rel

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)


def _intensities(spec, pr, w):
    """Oracle forward model on every frame, then the seeded Poisson counts; sqrt as float32."""
    f0 = ops.intensities(pr["u_true"], w, pr["offsets"])
    f = synthetic.poisson_counts(f0, spec.peak, pr["rng_poisson"]) if spec.peak else f0
    del f0
    return np.sqrt(f).astype(np.float32)


class _F:
    """f_j = sqrt_f_j^2 in FP64 for the frames asked for (the oracle's view of the bound data)."""

    def __init__(self, sf32, j0=0):
        self.sf32, self.j0 = sf32, j0

    def __getitem__(self, j):
        return self.sf32[self.j0 + j].astype(np.float64) ** 2


def _snapshot(st, subs, g, D0=0, J0=0, blind=False):
    """The parts of iterate n that the local step reads, in the oracle's (problem-local) indexing."""
    torch.cuda.synchronize()
    u_all = st.u_sub()
    u = [host(u_all[D0 + d]) for d in range(g.D)]
    lam = {(a - D0, b - D0): host(v) for (a, b), v in st.lam().items() if D0 <= a < D0 + g.D}
    js = sorted({int(j) for d in subs for j in g.frames_of[d]})
    idx = torch.tensor([J0 + j for j in js], device="cuda")
    G = host(st.gamma()[idx])
    gamma = {j: G[k] for k, j in enumerate(js)}
    out = dict(u=u, lam=lam, gamma=gamma)
    if blind:
        out["w_sub"] = list(host(st.probe_copies()))
        out["delta"] = list(host(st.probe_multipliers()))
    return out


def _compare(st, want, g, D0=0, J0=0, illum=None):
    """Relative errors of iterate n+1 on the chosen subdomains; u in the plain norm, or,
    with illum given, in the illumination-weighted norm ||A_d du|| / ||A_d u||
    (||A_d x||^2 = sum illum_d |x|^2, eq. AtA)."""
    torch.cuda.synchronize()
    u_all, lam_all, G_all = st.u_sub(), st.lam(), st.gamma()
    e = {}
    num = den = 0.0
    for d, ud in want["u"].items():
        got = host(u_all[D0 + d])
        wt = np.ones(got.shape) if illum is None else illum[d]
        num += np.sum(wt * np.abs(got - ud) ** 2)
        den += np.sum(wt * np.abs(ud) ** 2)
    e["u" if illum is None else "u_weighted"] = float(np.sqrt(num / den))
    js = sorted(want["gamma"])
    idx = torch.tensor([J0 + j for j in js], device="cuda")
    e["gamma"] = rel(host(G_all[idx]), np.stack([want["gamma"][j] for j in js]))
    e["lam"] = max(rel(host(lam_all[(a + D0, b + D0)]), v) for (a, b), v in want["lam"].items())
    if "w" in want:
        e["w"] = rel(host(st.probe()), want["w"])
        subs = sorted(want["w_sub"])
        e["w_sub"] = rel(host(st.probe_copies())[subs], np.stack([want["w_sub"][d] for d in subs]))
        e["delta"] = rel(host(st.probe_multipliers())[subs], np.stack([want["delta"][d] for d in subs]))
    return e


def _subs(g):
    """A corner, an edge and an interior subdomain of a grid partition."""
    D = g.D
    return sorted({0, min(D - 1, 3), D // 2 + (int(np.sqrt(D)) // 2 if D >= 9 else 0)})


@pytest.fixture(scope="module")
def c5_inputs():
    spec = synthetic.CONFIGS["c5"]
    pr = synthetic.draw_problem(spec)
    w_true = pr["w"].astype(np.complex64).astype(np.complex128)
    return spec, pr, w_true, _intensities(spec, pr, w_true)


@pytest.mark.parametrize("blind", [False, True], ids=["known_probe", "blind"])
def test_c5_full_size_one_iteration(blind, c5_inputs):
    spec, pr, w_true, sf32 = c5_inputs
    say("full size 2048^2 / 6561 frames, blind", blind)
    eta = 0.1
    plan = odp.Plan(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"], eps=0.5, eta=eta, r=1.0, mu=1.0,
                    blind=blind)
    g = build_geometry(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"])
    mean_energy = float(np.mean(np.sum(sf32.astype(np.float64) ** 2, axis=(1, 2))))
    w0 = (synthetic.make_probe(spec.p, spec.init_radius, 0.0)
          * synthetic.problems.blind_init_amplitude(mean_energy, spec.init_radius)).astype(np.complex64)
    plan.bind(dev_f32(sf32), dev_c64(w0 if blind else w_true))
    mu = 0.5 * eta * max(len(fr) for fr in g.frames_of)
    r = 0.5 * eta * plan.illum_max()
    plan.set_params(r=r, mu=mu)
    st = plan.new_state(w0=dev_c64(w0) if blind else None)
    plan.iterate(st, 2)
    subs = _subs(g)
    s = _snapshot(st, subs, g, blind=blind)
    plan.iterate(st, 1)
    f = _F(sf32)
    if blind:
        want = local.od2bp_step_local(g, f, s["u"], s["lam"], s["gamma"], s["w_sub"], s["delta"], 0.5, eta, r, mu,
                                      subs)
        # the U-step divides by the new copy's illumination, which falls to ~1e-6 of its
        # maximum at the frame corners: u is compared in the norm that illumination weights
        illum = {d: subdomain_illumination(g, want["w_sub"][d], d) for d in subs}
    else:
        want = local.od2pm_step_local(g, w_true, f, s["u"], s["lam"], s["gamma"], 0.5, eta, r, subs)
        illum = None
    e = _compare(st, want, g, illum=illum)
    say("full size errors", subs, e)
    assert max(e.values()) <= 1e-5, e       # one iteration: the operator bound


@pytest.fixture(scope="module")
def c4_batch():
    """The 64-problem batch as the benchmark runs it: one batch plan per probe size,
    bound, per-problem penalties, autotuned.  Returns [(plan, [(spec, pr, w, sqrt_f)])]."""
    specs = synthetic.batch_specs(64)
    eta = 0.1
    groups = {}
    for s in specs:
        groups.setdefault(s.p, []).append(s)
    out = []
    for p, group in sorted(groups.items()):
        probs, sfs, ws, data = [], [], [], []
        for s in group:
            pr = synthetic.draw_problem(s)
            w = pr["w"].astype(np.complex64).astype(np.complex128)
            sf = _intensities(s, pr, w)
            sfs.append(sf)
            ws.append(w)
            data.append((s, pr, w, sf))
            probs.append(dict(H=s.n, W=s.n, p=p, offsets=pr["offsets"], frame_sub=pr["frame_sub"], eps=0.5, eta=eta,
                              r=1.0))
        plan = odp.Plan.batch(probs)
        plan.bind(dev_f32(np.concatenate(sfs)), dev_c64(np.stack(ws)))
        plan.set_penalties([0.5 * eta * plan.entry(i).illum_max for i in range(len(group))])
        scratch = plan.new_state()
        t = plan.autotune(scratch, iters=3)
        say("batch p", p, "problems", len(group), "tuning", t.transform, t.xcd_slice, t.tiling)
        del scratch
        out.append((plan, data, t.transform))
    return out


def _split_bf16(transform):
    """The split-BF16 transforms (reading 18): one iteration within 1e-4 instead of 1e-5,
    and the oracle's sensitivity taken at a hi + lo pair's resolution (2^-17)."""
    return transform in (odp.ODP_DFT_SPLIT_BF16, odp.ODP_HYBRID_MFMA)


def test_c4_full_batch_one_problem_per_probe_size(c4_batch):
    say("full 64-problem batch")
    eta = 0.1
    plans, states, picks = [], [], []
    for plan, data, tr in c4_batch:
        # the problem with the most subdomains of this probe size
        i = max(range(len(data)), key=lambda q: plan.entry(q).D)
        picks.append((plan, i, data[i], tr))
        plans.append(plan)
        states.append(plan.new_state())
    odp.Graph(plans, states, 2).launch()
    snaps = []
    for (plan, i, (s, pr, w, sf), tr), st in zip(picks, states):
        e = plan.entry(i)
        g = build_geometry(s.n, s.n, s.p, pr["offsets"], pr["frame_sub"])
        subs = _subs(g)
        snaps.append((g, subs, _snapshot(st, subs, g, D0=e.D0, J0=e.J0)))
    odp.Graph(plans, states, 1).launch()
    for (plan, i, (s, pr, w, sf), tr), st, (g, subs, snap) in zip(picks, states, snaps):
        e = plan.entry(i)
        want = local.od2pm_step_local(g, w, _F(sf), snap["u"], snap["lam"], snap["gamma"], 0.5, eta, e.r, subs)
        err = _compare(st, want, g, D0=e.D0, J0=e.J0)
        say("batch p", s.p, "problem", i, "n", s.n, "D", g.D, "transform", tr, "errors", err)
        assert max(err.values()) <= (1e-4 if _split_bf16(tr) else 1e-5), err


def test_c4_batch_100_iterations_smallest_problems(c4_batch):
    """K = 100 iterations of the whole batch in one graph (the configuration's iteration
    count); the merged image of the smallest problem of each probe size against the FP64
    oracle's 100 iterations of that problem alone.  Bound max(1e-3, 2 s_100) on the Poisson
    data, s_100 the oracle's own distance after 100 iterations between runs whose sqrt(f)
    differs by half a float32 ulp (by 2^-17 if the autotuner chose a split-BF16 transform;
    the larger of two seeds; the reading of the K-iteration bound used for the 512^2
    workload)."""
    from oracle.od2p import merge, od2pm_run
    K, eta = 100, 0.1
    plans = [plan for plan, _, _ in c4_batch]
    states = [plan.new_state() for plan in plans]
    odp.Graph(plans, states, K).launch()
    torch.cuda.synchronize()
    for (plan, data, tr), st in zip(c4_batch, states):
        i = min(range(len(data)), key=lambda q: (plan.entry(q).J, q))
        s, pr, w, sf = data[i]
        e = plan.entry(i)
        g = build_geometry(s.n, s.n, s.p, pr["offsets"], pr["frame_sub"])
        img = host(plan.merge(st))[e.row0:e.row0 + e.H, e.col0:e.col0 + e.W]
        f = sf.astype(np.float64) ** 2
        ost, _ = od2pm_run(g, w, f, 0.5, eta, e.r, K)
        want = merge(g, ost.u)
        sens = 0.0
        for seed in (7, 8):
            unit = np.random.default_rng(seed).uniform(-1.0, 1.0, sf.shape)
            fp = (sf.astype(np.float64) * (1.0 + (2.0 ** -17 if _split_bf16(tr) else 2.0 ** -24) * unit)) ** 2
            op, _ = od2pm_run(g, w, fp, 0.5, eta, e.r, K)
            sens = max(sens, rel(merge(g, op.u), want))
        err = rel(img, want)
        bound = max(1e-3, 2.0 * sens)
        say("batch p", s.p, "transform", tr, "smallest problem", i, "J", e.J, "D", e.D, "n", s.n, f"K={K} err {err:.3e} "
            f"s_K {sens:.3e} bound {bound:.1e}")
        assert err <= bound, (err, bound)

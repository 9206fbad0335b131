"""GPU tests of the automatic overlap penalty (residual balancing on the consensus
constraints): the penalties the library picks, and the iterates, against the FP64
oracle's balanced runs."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import paper_2011_00162_amd as odp
from oracle import balance
from oracle.od2p import od2pm_run
from tests.gpu_util import dev_c64, dev_f32, gpu_plan, host, rel_list, rounded_inputs, same_state
from tests.oracle_problems import oracle_problem, tiny_spec

pytestmark = pytest.mark.gpu

# every check's ratio rp/rd stays this factor away from mu and 1/mu, so the GPU's
# residuals (FP32 iterates, FP64 sums) take the oracle's decisions
MARGIN = 1.03
PERIOD = 4


def say(*a):
    print("[gpu]", *a, flush=True)


def _balanced(P, K, mu):
    w, _, f = rounded_inputs(P)
    tr = []
    st, _, rh = balance.od2pm_run_balanced(P["geom"], w, f, P["eps"], P["eta"], P["r"], K, mu=mu, period=PERIOD,
                                           trace=tr)
    return st, rh, tr


def _clear(tr, mu):
    lm = math.log(mu)
    return all(abs(abs(math.log(rp / rd)) - lm) >= math.log(MARGIN) for _, rp, rd in tr
               if np.isfinite(rp) and np.isfinite(rd))


def _pick_mu(Ps, K):
    """The first mu whose oracle runs keep every check clear of both thresholds and
    change r at least once."""
    for mu in (10.0, 8.0, 6.0, 5.0, 4.0, 3.0):
        runs = [_balanced(P, K, mu) for P in Ps]
        if all(_clear(tr, mu) for _, _, tr in runs) and any(len(set(rh)) > 1 for _, rh, _ in runs):
            return mu, runs
    pytest.fail("no mu with margin")


def test_single_problem_penalties_follow_the_oracle():
    spec = tiny_spec(n=160, p=32, step=8, jitter=2, dy=1, dx=4, radius=12, peak=None)
    say("balance single")
    P = oracle_problem(spec)
    K = 24
    mu, [(ost, rh, _)] = _pick_mu([P], K)
    plan = gpu_plan(P)
    plan.set_balancing(mu, 2.0, PERIOD, 0)
    st = plan.new_state()
    got = []
    for _ in range(K // PERIOD):
        plan.iterate(st, PERIOD)
        got.append(plan.penalties()[0])
    want = rh[PERIOD - 1::PERIOD]
    say("balance r/r0", [g / P["r"] for g in got], "mu", mu)
    assert all(math.isclose(g, x, rel_tol=1e-12) for g, x in zip(got, want)), (got, want)
    assert len(set(got)) > 1
    assert rel_list([host(t) for t in st.u_sub()], ost.u) <= 1e-4


@pytest.mark.parametrize("p,transform", [(64, odp.ODP_FFT_F32), (64, odp.ODP_DFT_SPLIT_BF16), (128, odp.ODP_FFT_F32)],
                         ids=["p64_fft", "p64_split_bf16", "p128_two_half"])
def test_penalties_follow_the_oracle_with_the_larger_frame_sweeps(p, transform):
    """The residual sums come from the statistics variants of every sweep kernel."""
    q = p // 4
    spec = tiny_spec(n=3 * p, p=p, step=q, jitter=2, dy=2, dx=2, radius=3 * p // 8, peak=None)
    say("balance single, p", p, "transform", transform)
    P = oracle_problem(spec)
    K = 24
    mu, [(ost, rh, _)] = _pick_mu([P], K)
    w, sf32, _ = rounded_inputs(P)
    plan = odp.Plan(spec.n, spec.n, p, P["pr"]["offsets"], P["pr"]["frame_sub"], eps=P["eps"], eta=P["eta"],
                    r=P["r"], transform=transform)
    plan.bind(dev_f32(sf32), dev_c64(w))
    plan.set_balancing(mu, 2.0, PERIOD, 0)
    st = plan.new_state()
    got = []
    for _ in range(K // PERIOD):
        plan.iterate(st, PERIOD)
        got.append(plan.penalties()[0])
    want = rh[PERIOD - 1::PERIOD]
    say("balance r/r0", [g / P["r"] for g in got], "mu", mu)
    assert all(math.isclose(g, x, rel_tol=1e-12) for g, x in zip(got, want)), (got, want)
    assert len(set(got)) > 1
    # the K-iteration reconstruction bound
    assert rel_list([host(t) for t in st.u_sub()], ost.u) <= 1e-3


def test_batch_penalties_adapt_per_problem_and_graphs_refuse():
    say("balance batch")
    specs = [tiny_spec(n=128, p=32, step=8, jitter=1, dy=2, dx=2, radius=12, peak=1e4, seed=41),
             tiny_spec(n=160, p=32, step=8, jitter=2, dy=1, dx=4, radius=12, peak=None, seed=42),
             tiny_spec(n=96, p=32, step=8, jitter=1, dy=1, dx=1, radius=12, peak=1e4, seed=43)]
    Ps = [oracle_problem(s) for s in specs]
    K = 16
    mu, runs = _pick_mu(Ps, K)
    plan = odp.Plan.batch([dict(H=P["pr"]["spec"].n, W=P["pr"]["spec"].n, p=32, offsets=P["pr"]["offsets"],
                                frame_sub=P["pr"]["frame_sub"], r=P["r"]) for P in Ps])
    plan.bind(dev_f32(np.concatenate([rounded_inputs(P)[1] for P in Ps])),
              dev_c64(np.stack([rounded_inputs(P)[0] for P in Ps])))
    plan.set_balancing(mu, 2.0, PERIOD, 0)
    st = plan.new_state()
    with pytest.raises(odp.OdpError):
        odp.Graph([plan], [st], 2)                  # host-driven: not capturable
    plan.iterate(st, K)
    got = plan.penalties()
    for i, ((ost, rh, _), P) in enumerate(zip(runs, Ps)):
        assert math.isclose(got[i], rh[-1], rel_tol=1e-12), (i, got[i], rh[-1])
        e = plan.entry(i)
        # the K-iteration reconstruction bound
        assert rel_list([host(t) for t in st.u_sub()[e.D0:e.D0 + e.D]], ost.u) <= 1e-3, i
    assert got[2] == Ps[2]["r"]                     # one subdomain: nothing to balance


def test_balancing_off_and_until():
    spec = tiny_spec(n=128, p=32, step=8, jitter=1, dy=2, dx=2, radius=12, peak=1e4)
    say("balance off / until")
    P = oracle_problem(spec)
    plan = gpu_plan(P)
    plan.set_balancing(np.inf, 2.0, 1, 0)           # checks every iteration, never triggers
    a = plan.new_state()
    plan.iterate(a, 6)
    assert plan.penalties() == [P["r"]]
    plan.set_balancing(10.0, 2.0, 0, 0)             # off
    b = plan.new_state()
    plan.iterate(b, 6, stats=True)
    assert same_state(a, b)
    w, _, f = rounded_inputs(P)
    tr = []
    _, _, rh = balance.od2pm_run_balanced(P["geom"], w, f, P["eps"], P["eta"], P["r"], 12, mu=1.0, period=1,
                                          until=3, trace=tr)
    assert _clear(tr, 1.0)
    plan.set_params(r=P["r"])
    plan.set_balancing(1.0, 2.0, 1, 3)              # mu = 1: a change at each of the first 3
    c = plan.new_state()
    plan.iterate(c, 12)
    assert math.isclose(plan.penalties()[0], rh[-1], rel_tol=1e-12)
    assert rh[2] != P["r"] and rh[3:] == [rh[2]] * 9


def _balanced_both(P, K, mu, which):
    w, _, f = rounded_inputs(P)
    tr, tre, eh = [], [], []
    st, _, rh = balance.od2pm_run_balanced(P["geom"], w, f, P["eps"], P["eta"], P["r"], K, mu=mu, period=PERIOD,
                                           trace=tr, trace_eta=tre, eta_hist=eh,
                                           balance_r=bool(which & odp.ODP_BALANCE_R),
                                           balance_eta=bool(which & odp.ODP_BALANCE_ETA))
    return st, rh, eh, tr + tre


@pytest.mark.parametrize("which", [2, 3], ids=["eta", "r_and_eta"])
def test_data_penalty_follows_the_oracle(which):
    # noise-free data: on Poisson data the iteration amplifies the FP32 rounding beyond the
    # 1e-4 compared here within these 24 iterations, with or without balancing
    spec = tiny_spec(n=160, p=32, step=8, jitter=2, dy=1, dx=4, radius=12, peak=None)
    say("balance eta, which", which)
    P = oracle_problem(spec)
    K = 24
    for mu in (10.0, 8.0, 6.0, 5.0, 4.0, 3.0, 2.0):
        ost, rh, eh, tr = _balanced_both(P, K, mu, which)
        if _clear(tr, mu) and len(set(eh)) > 1:
            break
    else:
        pytest.fail("no mu with margin")
    plan = gpu_plan(P)
    plan.set_balancing(mu, 2.0, PERIOD, 0, which)
    st = plan.new_state()
    got_r, got_eta = [], []
    for _ in range(K // PERIOD):
        plan.iterate(st, PERIOD)
        got_r.append(plan.penalties()[0])
        got_eta.append(plan.eta())
    say("balance eta/eta0", [e / P["eta"] for e in got_eta], "r/r0", [r / P["r"] for r in got_r], "mu", mu)
    assert all(math.isclose(g, x, rel_tol=1e-12) for g, x in zip(got_eta, eh[PERIOD - 1::PERIOD])), (got_eta, eh)
    assert all(math.isclose(g, x, rel_tol=1e-12) for g, x in zip(got_r, rh[PERIOD - 1::PERIOD])), (got_r, rh)
    assert rel_list([host(t) for t in st.u_sub()], ost.u) <= 1e-4


def test_data_penalty_refused_for_blind_plans():
    spec = tiny_spec(n=128, p=32, step=8, jitter=1, dy=2, dx=2, radius=12, peak=1e4)
    P = oracle_problem(spec)
    mu = 0.5 * P["eta"] * max(len(fr) for fr in P["geom"].frames_of)
    plan = gpu_plan(P, blind=True, mu=mu)
    with pytest.raises(odp.OdpError):
        plan.set_balancing(10.0, 2.0, 4, 0, odp.ODP_BALANCE_ETA)
    plan.set_balancing(10.0, 2.0, 4, 0, odp.ODP_BALANCE_R)   # r stays available


def test_autotune_leaves_the_penalties_and_restores_balancing():
    spec = tiny_spec(n=128, p=32, step=8, jitter=1, dy=2, dx=2, radius=12, peak=1e4)
    say("balancing across autotune")
    P = oracle_problem(spec)
    plan = gpu_plan(P)
    plan.set_balancing(1.0, 2.0, 1, 0)              # mu = 1: every check changes r
    plan.autotune(plan.new_state(), iters=2)
    assert plan.penalties() == [P["r"]]             # timed with balancing off
    st = plan.new_state()
    plan.iterate(st, 1)
    assert plan.penalties() != [P["r"]]             # and on again afterwards


def _eight_problem_batch():
    """Eight small known-probe problems with subdomain pairs (the residual sums hold NRES
    doubles per problem, so eight problems reach well past any alignment padding)."""
    specs = [tiny_spec(n=96 + 16 * (i % 3), p=32, step=8, jitter=1, dy=1 + i % 2, dx=2, radius=12,
                       peak=None if i % 2 else 1e4, seed=60 + i) for i in range(8)]
    Ps = [oracle_problem(s) for s in specs]
    plan = odp.Plan.batch([dict(H=P["pr"]["spec"].n, W=P["pr"]["spec"].n, p=32, offsets=P["pr"]["offsets"],
                                frame_sub=P["pr"]["frame_sub"], r=P["r"]) for P in Ps])
    return Ps, plan


def test_residual_sums_stay_inside_the_workspace():
    """Balancing r and eta on eight problems writes every problem's residual sums inside the
    workspace: a guard region right after workspace_bytes keeps its fill pattern."""
    say("balance: workspace guard, 8 problems")
    Ps, plan = _eight_problem_batch()
    nb = plan.info.workspace_bytes
    buf = torch.full((nb + 4096,), 0xA5, dtype=torch.uint8, device="cuda")
    plan.bind(dev_f32(np.concatenate([rounded_inputs(P)[1] for P in Ps])),
              dev_c64(np.stack([rounded_inputs(P)[0] for P in Ps])), workspace=buf)
    plan.set_balancing(1.0, 2.0, 1, 0, odp.ODP_BALANCE_R | odp.ODP_BALANCE_ETA)   # mu = 1: checks act
    st = plan.new_state()
    plan.iterate(st, 6)
    torch.cuda.synchronize()
    assert bool((buf[nb:] == 0xA5).all()), "residual sums written past the workspace"
    assert plan.eta() != 0.1 and len(set(plan.penalties())) > 1
    assert all(bool(torch.isfinite(torch.view_as_real(t)).all()) for t in st.u_sub())


def test_stopped_problems_take_no_part_in_balancing():
    """After every problem of a batch has met its iteration cap, further balanced iterations
    change neither the penalties nor any bit of the state (r and eta both balanced)."""
    say("balance: stopped problems frozen")
    Ps, plan = _eight_problem_batch()
    plan.bind(dev_f32(np.concatenate([rounded_inputs(P)[1] for P in Ps])),
              dev_c64(np.stack([rounded_inputs(P)[0] for P in Ps])))
    plan.set_stopping(odp.ODP_STOP_NONE, 0.0, 4)
    plan.set_balancing(1.0, 2.0, 1, 0, odp.ODP_BALANCE_R | odp.ODP_BALANCE_ETA)
    st = plan.new_state()
    plan.iterate(st, 4)
    assert all(s["stopped"] for s in plan.stop_status(st))
    r0, eta0, frozen = plan.penalties(), plan.eta(), st.clone()
    plan.iterate(st, 4)
    assert plan.penalties() == r0 and plan.eta() == eta0
    assert same_state(st, frozen)

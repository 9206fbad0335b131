"""GPU tests of the device-side stopping rules (Sec. 4): each problem of a plan stops
after the first iteration whose measure meets the tolerance, or at the iteration cap;
its state then stays that iterate while the other problems go on, in eager calls and
inside a graph.  The stop points come from the FP64 oracle's trajectories."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import synthetic
import paper_2011_00162_amd as odp
from oracle.od2p import od2pm_run
from tests.gpu_util import dev_c64, dev_f32, gpu_plan, host, rel, rel_list, rounded_inputs, same_state
from tests.oracle_problems import oracle_problem, tiny_spec

pytestmark = pytest.mark.gpu

# the tolerance sits at least this factor away from every measure the decision reads,
# so the FP32 measures (within about 1e-3 of the oracle's) take the same decisions
MARGIN = 1.05


def say(*a):
    print("[gpu]", *a, flush=True)


def _pick_tol(seqs, first=2, after=3, all_stop=True):
    """(tol, stop indices): tol between two consecutive distinct values of all sequences,
    at least MARGIN from both; per sequence the first index m with value <= tol,
    first <= m < len - after (so iterations remain after the stop), or None where no
    value is <= tol (allowed unless all_stop).  Among the candidates, the one giving the
    most distinct outcomes, then the latest first stop."""
    vals = sorted({float(v) for s in seqs for v in s}, reverse=True)
    best = None
    for a, b in zip(vals, vals[1:]):
        if not (b > 0 and a / b >= MARGIN ** 2):
            continue
        tol = math.sqrt(a * b)
        ms = []
        for s in seqs:
            hit = [k for k, v in enumerate(s) if v <= tol]
            if (not hit and all_stop) or (hit and not first <= hit[0] < len(s) - after):
                break
            ms.append(hit[0] if hit else None)
        else:
            stops = [m for m in ms if m is not None]
            if not stops:
                continue
            key = (len(set(ms)), min(stops))
            if best is None or key > best[0]:
                best = (key, tol, ms)
    assert best is not None, "no tolerance with margin"
    return best[1], best[2]


def _oracle_run(P, K):
    w, _, f = rounded_inputs(P)
    return od2pm_run(P["geom"], w, f, P["eps"], P["eta"], P["r"], K)


@pytest.mark.parametrize("measure,peak", [(odp.ODP_STOP_RE, 1e4), (odp.ODP_STOP_RF, None)], ids=["RE_noisy", "RF_clean"])
def test_single_problem_stops_where_the_oracle_does(measure, peak):
    spec = tiny_spec(n=128, p=32, step=8, jitter=1, dy=1, dx=2, radius=12, peak=peak)
    say("stop single", measure)
    P = oracle_problem(spec)
    K = 16
    _, hist = _oracle_run(P, K)
    key = "RE" if measure == odp.ODP_STOP_RE else "RF"
    tol, (m,) = _pick_tol([[h[key] for h in hist]])
    plan = gpu_plan(P)
    plan.set_stopping(measure, tol, 0)
    st = plan.new_state()
    assert plan.stop_status(st)[0] == dict(iters=0, stopped=False, rf=0.0, re=0.0, g=0.0)
    plan.iterate(st, K)
    s = plan.stop_status(st)[0]
    assert (s["iters"], s["stopped"]) == (m + 1, True), (s, m)
    assert abs(s["rf"] - hist[m]["RF"]) <= 1e-3 * hist[m]["RF"]
    assert abs(s["re"] - hist[m]["RE"]) <= 1e-3 * hist[m]["RE"]
    ost, _ = _oracle_run(P, m + 1)
    assert rel_list([host(t) for t in st.u_sub()], ost.u) <= 1e-4
    # the stopped state is exactly the iterate of m + 1 iterations (the rule off)
    plan.set_stopping(odp.ODP_STOP_NONE, 0.0, 0)
    ref = plan.new_state()
    plan.iterate(ref, m + 1, stats=True)
    assert same_state(st, ref)


def test_iteration_cap_and_state_init_reset():
    spec = tiny_spec(n=128, p=32, step=8, jitter=1, dy=2, dx=2, radius=12, peak=1e4)
    say("stop cap")
    P = oracle_problem(spec)
    plan = gpu_plan(P)
    plan.set_stopping(odp.ODP_STOP_NONE, 0.0, 3)
    st = plan.new_state()
    plan.iterate(st, 5)
    s = plan.stop_status(st)[0]
    assert (s["iters"], s["stopped"]) == (3, True)
    plan.set_stopping(odp.ODP_STOP_NONE, 0.0, 0)
    ref = plan.new_state()
    plan.iterate(ref, 3, stats=True)
    assert same_state(st, ref)
    assert plan.stop_status(ref)[0]["iters"] == 0          # no rule: no progress kept
    plan.set_stopping(odp.ODP_STOP_NONE, 0.0, 3)
    from paper_2011_00162_amd._lib import lib
    assert lib().odp_state_init(plan._h, st.buf.data_ptr(), None, None) == 0
    assert plan.stop_status(st)[0]["iters"] == 0           # init clears the progress
    plan.iterate(st, 4)
    assert same_state(st, ref)


def test_blind_problem_freezes_probe_and_image():
    spec = tiny_spec(n=128, p=32, step=8, jitter=1, dy=2, dx=2, radius=12, peak=1e4)
    say("stop blind")
    P = oracle_problem(spec)
    g = P["geom"]
    mu = 0.5 * P["eta"] * max(len(fr) for fr in g.frames_of)
    plan = gpu_plan(P, blind=True, mu=mu)
    w0 = plan.blind_initial_probe()
    plan.set_stopping(odp.ODP_STOP_RF, 0.0, 2)              # RF > 0 here: the cap decides
    st = plan.new_state(w0=w0)
    plan.iterate(st, 4)
    s = plan.stop_status(st)[0]
    assert (s["iters"], s["stopped"]) == (2, True)
    plan.set_stopping(odp.ODP_STOP_NONE, 0.0, 0)
    ref = plan.new_state(w0=w0)
    plan.iterate(ref, 2, stats=True)
    assert same_state(st, ref)                             # u, Gamma, Lam, w, w_d, Delta


def _batch_items():
    # uneven sizes, partitions and noise: their RE trajectories fall at different rates
    shapes = [(128, 8, 1, 1, 2, 1e4, 31), (96, 6, 1, 2, 1, 1e5, 33), (160, 8, 2, 2, 3, 1e3, 35)]
    out = []
    for n, step, jit, dy, dx, peak, seed in shapes:
        P = oracle_problem(tiny_spec(n=n, p=32, step=step, jitter=jit, dy=dy, dx=dx, radius=12, peak=peak,
                                     seed=seed))
        out.append(P)
    return out


def test_batch_problems_stop_independently_also_in_a_graph():
    say("stop batch")
    items = _batch_items()
    K = 14
    runs = [_oracle_run(P, K)[1] for P in items]
    tol, ms = _pick_tol([[h["RE"] for h in hist] for hist in runs], all_stop=False)
    want = [(K, False) if m is None else (m + 1, True) for m in ms]
    say("stop batch tol", tol, "iterations, stopped", want)
    assert len({m for m in ms}) >= 2                   # the problems do not all stop together
    plan = odp.Plan.batch([dict(H=P["pr"]["spec"].n, W=P["pr"]["spec"].n, p=32, offsets=P["pr"]["offsets"],
                                frame_sub=P["pr"]["frame_sub"], r=P["r"]) for P in items])
    sf = np.concatenate([rounded_inputs(P)[1] for P in items])
    w = np.stack([rounded_inputs(P)[0] for P in items])
    plan.bind(dev_f32(sf), dev_c64(w))
    plan.set_stopping(odp.ODP_STOP_RE, tol, 0)
    a = plan.new_state()
    plan.iterate(a, K)
    stat = plan.stop_status(a)
    assert [(s["iters"], s["stopped"]) for s in stat] == want, (stat, ms)
    for i, (P, (n_it, _)) in enumerate(zip(items, want)):
        e = plan.entry(i)
        ost, _ = _oracle_run(P, n_it)
        # the K-iteration reconstruction bound (a noisy problem runs all K here)
        assert rel_list([host(t) for t in a.u_sub()[e.D0:e.D0 + e.D]], ost.u) <= 1e-3, i
    # a graph of K iterations gives the same outcome and states; on a second replay (eager
    # work in between) the stopped problems stay as they are and the others go on
    b = plan.new_state()
    gr = odp.Graph([plan], [b], K)
    gr.launch()
    torch.cuda.synchronize()
    assert plan.stop_status(b) == stat
    assert same_state(a, b)
    c = b.clone()
    gr.launch()
    torch.cuda.synchronize()
    after = plan.stop_status(b)
    for i, (_, stopped) in enumerate(want):
        e = plan.entry(i)
        same_u = all(torch.equal(x, y) for x, y in zip(b.u_sub()[e.D0:e.D0 + e.D], c.u_sub()[e.D0:e.D0 + e.D]))
        same_g = torch.equal(b.gamma()[e.J0:e.J0 + e.J], c.gamma()[e.J0:e.J0 + e.J])
        if stopped:
            assert after[i] == stat[i] and same_u and same_g, i
        else:
            assert after[i]["iters"] > K and not same_u, i


def _cap_freezes(plan, cap=2, extra=2, w0=None):
    """With the rule off but an iteration cap, a longer run stops at the cap and equals a
    run of exactly that many iterations (statistics variants on both sides)."""
    plan.set_stopping(odp.ODP_STOP_NONE, 0.0, cap)
    st = plan.new_state(w0=w0)
    plan.iterate(st, cap + extra)
    assert [(s["iters"], s["stopped"]) for s in plan.stop_status(st)] == [(cap, True)] * plan.n_problems()
    plan.set_stopping(odp.ODP_STOP_NONE, 0.0, 0)
    ref = plan.new_state(w0=w0)
    plan.iterate(ref, cap, stats=True)
    assert same_state(st, ref)


def test_cap_with_the_mfma_transform():
    """The split-BF16 sweep's persistent loop skips a stopped problem's frames."""
    spec = tiny_spec(n=192, p=64, step=16, jitter=2, dy=2, dx=2, radius=24, peak=1e4)
    say("stop cap, split-BF16 transform")
    P = oracle_problem(spec)
    w, sf32, _ = rounded_inputs(P)
    plan = odp.Plan(spec.n, spec.n, 64, P["pr"]["offsets"], P["pr"]["frame_sub"], r=P["r"],
                    transform=odp.ODP_DFT_SPLIT_BF16)
    plan.bind(dev_f32(sf32), dev_c64(w))
    _cap_freezes(plan)


@pytest.mark.parametrize("blind", [False, True], ids=["known_probe", "blind"])
def test_cap_with_the_two_half_transform(blind):
    """The p = 128 sweep (one frame per workgroup, two half passes) and, blind, the probe
    copies skip a stopped problem's frames too."""
    spec = tiny_spec(n=256, p=128, step=32, jitter=2, dy=2, dx=2, radius=48, peak=1e3)
    say("stop cap, p = 128, blind", blind)
    P = oracle_problem(spec)
    mu = 0.5 * P["eta"] * max(len(fr) for fr in P["geom"].frames_of) if blind else 0.0
    plan = gpu_plan(P, blind=blind, mu=mu)
    _cap_freezes(plan, w0=plan.blind_initial_probe() if blind else None)


def test_cap_with_five_to_eight_copies():
    """Cells with five or more copies (the general pixel kernel) also stop."""
    from oracle.geometry import build_geometry
    spec = tiny_spec(n=96, p=32, step=8, jitter=1, radius=12, peak=1e4)
    say("stop cap, six copies per pixel")
    P = oracle_problem(spec)
    pr = P["pr"]
    pr["frame_sub"] = (np.arange(len(pr["offsets"])) % 6).astype(np.int32)
    g = build_geometry(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"])
    from oracle.od2p import subdomain_illumination
    r = 0.5 * 0.1 * max(float(subdomain_illumination(g, pr["w"], d).max()) for d in range(g.D))
    plan = gpu_plan(P, r=r)
    assert plan.info.max_cover == 6
    _cap_freezes(plan)


@pytest.mark.parametrize("blind", [False, True], ids=["known_probe", "blind"])
@pytest.mark.parametrize("groups", [6, 12], ids=["six_copies", "twelve_copies"])
def test_statistics_variants_keep_the_iterate_with_many_copies(groups, blind):
    """The general pixel kernel (cells with 5-8 and 9-16 copies) forms u and Lam partner by
    partner without statistics and from whole partner arrays with them; both keep the same
    arithmetic order, so K iterations give the same state bit for bit either way."""
    from tests.test_gpu_streaming import _parts, _start
    spec = tiny_spec(n=96, p=32, step=8, jitter=1, radius=12, peak=1e4)
    say("statistics on/off,", groups, "subdomains interleaved,", "blind" if blind else "known probe")
    P = oracle_problem(spec)
    P["pr"]["frame_sub"] = (np.arange(len(P["pr"]["offsets"])) % groups).astype(np.int32)
    runs = []
    for stats in (False, True):
        plan = gpu_plan(P, r=1.0, blind=blind, mu=4.0 if blind else 0.0)
        assert plan.info.max_cover > (8 if groups > 8 else 4), plan.info.max_cover
        st = _start(plan, P, blind)
        plan.iterate(st, 4, stats=stats)
        torch.cuda.synchronize()
        runs.append(_parts(plan, st))
    a, b = runs
    differ = {k: int((a[k] != b[k]).sum()) for k in a if not torch.equal(a[k], b[k])}
    assert not differ, differ


def test_check_interval_stops_at_the_next_check():
    """every = 4: the rule is read after iterations 4, 8, ...; the problem stops at the
    first of those whose measure meets the tolerance, and the counts stay exact."""
    spec = tiny_spec(n=128, p=32, step=8, jitter=1, dy=1, dx=2, radius=12, peak=1e4)
    say("stop every 4")
    P = oracle_problem(spec)
    K, every = 24, 4
    _, hist = _oracle_run(P, K)
    checked = [hist[n]["RE"] for n in range(every - 1, K, every)]
    tol, (mc,) = _pick_tol([checked], first=1, after=1)
    n_stop = (mc + 1) * every
    plan = gpu_plan(P)
    plan.set_stopping(odp.ODP_STOP_RE, tol, 0, every)
    st = plan.new_state()
    plan.iterate(st, K)
    s = plan.stop_status(st)[0]
    assert (s["iters"], s["stopped"]) == (n_stop, True), (s, n_stop)
    assert abs(s["re"] - hist[n_stop - 1]["RE"]) <= 1e-3 * hist[n_stop - 1]["RE"]
    ost, _ = _oracle_run(P, n_stop)
    assert rel_list([host(t) for t in st.u_sub()], ost.u) <= 1e-4
    plan.set_stopping(odp.ODP_STOP_NONE, 0.0, 0)
    ref = plan.new_state()
    plan.iterate(ref, n_stop)          # the statistics variants change no bit of the iterate
    assert same_state(st, ref)
    plan.set_stopping(odp.ODP_STOP_RE, tol, 0, every)
    # a graph needs a whole number of check intervals
    with pytest.raises(odp.OdpError):
        odp.Graph([plan], [plan.new_state()], 6)
    b = plan.new_state()
    odp.Graph([plan], [b], 8).launch()
    torch.cuda.synchronize()
    assert plan.stop_status(b)[0]["iters"] == 8


def test_blind_re_rule_stops_where_the_oracle_does():
    """Algorithm 3 with the RE rule (Sec. 4) read after each iteration, against the FP64
    blind trajectory from the same start (the initial probe of the extended tests)."""
    from oracle import blind
    spec = tiny_spec(n=128, p=32, step=8, jitter=1, dy=2, dx=2, radius=12, peak=None)
    say("stop blind RE")
    P = oracle_problem(spec)
    g = P["geom"]
    w_true, sf32, f = rounded_inputs(P)
    mu = 0.5 * P["eta"] * max(len(fr) for fr in g.frames_of)
    plan = gpu_plan(P, blind=True, mu=mu)
    w0 = plan.blind_initial_probe()
    w0h = host(w0)
    K = 16
    _, hist = blind.od2bp_run(g, f, w0h, P["eps"], P["eta"], P["r"], mu, K)
    tol, (m,) = _pick_tol([[h["RE"] for h in hist]])
    plan.set_stopping(odp.ODP_STOP_RE, tol, 0)
    st = plan.new_state(w0=w0)
    plan.iterate(st, K)
    s = plan.stop_status(st)[0]
    assert (s["iters"], s["stopped"]) == (m + 1, True), (s, m)
    assert abs(s["re"] - hist[m]["RE"]) <= 1e-3 * hist[m]["RE"]
    ost, _ = blind.od2bp_run(g, f, w0h, P["eps"], P["eta"], P["r"], mu, m + 1)
    assert rel(host(st.probe()), ost.w) <= 1e-4
    plan.set_stopping(odp.ODP_STOP_NONE, 0.0, 0)
    ref = plan.new_state(w0=w0)
    plan.iterate(ref, m + 1)
    assert same_state(st, ref)


def test_autotune_restores_the_rule():
    """The autotuner times whole iterations with the rule off and puts it back."""
    spec = tiny_spec(n=128, p=32, step=8, jitter=1, dy=2, dx=2, radius=12, peak=1e4)
    say("stop rule across autotune")
    P = oracle_problem(spec)
    plan = gpu_plan(P)
    plan.set_stopping(odp.ODP_STOP_NONE, 0.0, 3)
    plan.autotune(plan.new_state(), iters=2)
    st = plan.new_state()
    plan.iterate(st, 5)
    assert [(s["iters"], s["stopped"]) for s in plan.stop_status(st)] == [(3, True)]

"""GPU tests of batched plans (many independent problems of uneven size in one
plan), graph replay and the autotuner."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import synthetic
import paper_2011_00162_amd as odp
from oracle import operators as ops
from oracle.geometry import build_geometry
from oracle.od2p import merge, od2pm_run, subdomain_illumination
from tests.gpu_util import dev_c64, dev_f32, host, rel, rel_list, same_state

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)


def _uneven_problems():
    """Four p = 64 problems of different image size, step, jitter, partition and noise."""
    shapes = [(192, 16, 2, 2, 2, 1e4), (256, 20, 1, 3, 2, None), (224, 24, 0, 2, 3, 1e3), (320, 18, 2, 4, 4, 1e5)]
    out = []
    for i, (n, step, jit, dy, dx, peak) in enumerate(shapes):
        spec = synthetic.ProblemSpec(f"b{i}", n=n, sigma=6.0, p=64, radius=24, quad=0.02, step=step, jitter=jit,
                                     dy=dy, dx=dx, peak=peak, iters=10, seed=100 + i)
        pr = synthetic.draw_problem(spec)
        w = pr["w"].astype(np.complex64).astype(np.complex128)
        f = synthetic.poisson_counts(ops.intensities(pr["u_true"], w, pr["offsets"]), peak, pr["rng_poisson"])
        sf32 = np.sqrt(f).astype(np.float32)
        g = build_geometry(n, n, 64, pr["offsets"], pr["frame_sub"])
        r = 0.5 * 0.1 * max(float(subdomain_illumination(g, w, d).max()) for d in range(g.D))
        out.append(dict(spec=spec, pr=pr, w=w, sf32=sf32, f=sf32.astype(np.float64) ** 2, g=g, r=r))
    return out


def _batch(items, transform=odp.ODP_FFT_F32):
    plan = odp.Plan.batch([dict(H=it["spec"].n, W=it["spec"].n, p=64, offsets=it["pr"]["offsets"],
                                frame_sub=it["pr"]["frame_sub"], r=it["r"], transform=transform) for it in items])
    sf = np.concatenate([it["sf32"] for it in items])
    w = np.stack([it["w"] for it in items])
    plan.bind(dev_f32(sf), dev_c64(w))
    return plan


def _member_u(plan, state, i):
    e = plan.entry(i)
    return [host(t) for t in state.u_sub()[e.D0:e.D0 + e.D]]


def test_batch_equals_individual_plans_bit_for_bit():
    say("batch vs individual plans")
    items = _uneven_problems()
    plan = _batch(items)
    st = plan.new_state()
    plan.iterate(st, 5)
    for i, it in enumerate(items):
        s = it["spec"]
        single = odp.Plan(s.n, s.n, 64, it["pr"]["offsets"], it["pr"]["frame_sub"], r=it["r"])
        single.bind(dev_f32(it["sf32"]), dev_c64(it["w"]))
        ss = single.new_state()
        single.iterate(ss, 5)
        got, want = _member_u(plan, st, i), [host(t) for t in ss.u_sub()]
        assert all(np.array_equal(a, b) for a, b in zip(got, want)), i
        e = plan.entry(i)
        assert torch.equal(st.gamma()[e.J0:e.J0 + e.J], ss.gamma())


def test_batch_member_matches_oracle_and_merge():
    say("batch member vs oracle")
    items = _uneven_problems()
    plan = _batch(items)
    st = plan.new_state()
    K = 8
    plan.iterate(st, K)
    img = host(plan.merge(st))
    for i in (1, 3):
        it = items[i]
        ost, _ = od2pm_run(it["g"], it["w"], it["f"], 0.5, 0.1, it["r"], K)
        assert rel_list(_member_u(plan, st, i), ost.u) <= 1e-4
        e = plan.entry(i)
        sub_img = img[e.row0:e.row0 + e.H, e.col0:e.col0 + e.W]
        assert rel(sub_img, merge(it["g"], ost.u)) <= 1e-4


def test_graph_replay_equals_direct_iterations():
    say("graph replay")
    items = _uneven_problems()
    plan = _batch(items)
    a = plan.new_state()
    plan.iterate(a, 6)
    b = plan.new_state()
    g = odp.Graph([plan], [b], 3)
    g.launch()
    torch.cuda.synchronize()
    g.launch()            # two replays = six iterations, eager work in between
    assert same_state(a, b)


def test_autotune_keeps_results_within_tolerance():
    say("autotune")
    items = _uneven_problems()
    plan = _batch(items)
    scratch = plan.new_state()
    t = plan.autotune(scratch, iters=3)
    say("autotune choice", dict(transform=t.transform, xcd_slice=t.xcd_slice, tile=(t.tile_rows, t.tile_cols),
                                ms=t.ms_per_iter, tried=t.n_tried))
    assert t.n_tried == 27 and t.ms_per_iter > 0     # 3 transforms x 3 placements x 3 tilings at p = 64
    st = plan.new_state()
    K = 8
    plan.iterate(st, K)
    it = items[2]
    ost, _ = od2pm_run(it["g"], it["w"], it["f"], 0.5, 0.1, it["r"], K)
    assert rel_list(_member_u(plan, st, 2), ost.u) <= 1e-3
    # every tiling and placement gives the same iterates (they only change the work split)
    plan.set_tuning(odp.ODP_FFT_F32, 1, 0)
    s0 = plan.new_state()
    plan.iterate(s0, 3)
    for xcd, tiling in ((0, 1), (0, 2), (2, 0), (2, 1), (2, 2)):
        plan.set_tuning(odp.ODP_FFT_F32, xcd, tiling)
        s1 = plan.new_state()
        plan.iterate(s1, 3)
        assert same_state(s0, s1), (xcd, tiling)


def test_per_problem_penalties():
    say("per-problem penalties")
    items = _uneven_problems()
    plan = _batch(items)
    r = [0.3 * it["r"] for it in items]
    plan.set_penalties(r)
    st = plan.new_state()
    plan.iterate(st, 4)
    it = items[0]
    ost, _ = od2pm_run(it["g"], it["w"], it["f"], 0.5, 0.1, r[0], 4)
    assert rel_list(_member_u(plan, st, 0), ost.u) <= 1e-4


def test_graph_refused_once_stale():
    """A graph keeps its plans' launch arguments and tables from capture: after a penalty,
    tuning or autotune change on one of them, launching it is refused until it is made again."""
    say("stale graph")
    items = _uneven_problems()[:2]
    plan = _batch(items)
    st = plan.new_state()
    g = odp.Graph([plan], [st], 2)
    g.launch()
    plan.set_penalties([it["r"] * 2.0 for it in items])
    with pytest.raises(odp.OdpError, match="stale"):
        g.launch()
    g = odp.Graph([plan], [st], 2)
    g.launch()
    t = plan.tuning()
    plan.set_tuning(t.transform, t.xcd_slice, t.tiling)     # unchanged: still valid
    g.launch()
    plan.set_tuning(t.transform, t.xcd_slice, (t.tiling + 1) % 3)
    with pytest.raises(odp.OdpError, match="stale"):
        g.launch()
    g = odp.Graph([plan], [st], 2)
    plan.autotune(plan.new_state(), iters=1)
    with pytest.raises(odp.OdpError, match="stale"):
        g.launch()
    torch.cuda.synchronize()

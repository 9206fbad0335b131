"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (FP32 kernels against FP64 on identical FP32-rounded inputs):
  operators (A, A*, A*A, prox)                      relative <= 1e-5
  one ADMM iteration from an arbitrary state          relative <= 1e-5, in norm and element
                                                      by element (tests.gpu_util: each value
                                                      at the scale of the operands its FP32
                                                      arithmetic combines)
  reconstruction after K iterations (merged image)    relative <= 1e-3
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import synthetic
import paper_2011_00162_amd as odp
from oracle import operators as ops, stagm
from oracle.geometry import build_geometry
from oracle.od2p import init_state, merge, od2pm_run, od2pm_step, subdomain_illumination
from tests.gpu_util import (dev_c64, dev_f32, gamma_elem_err, gpu_plan, host, lam_elem_err, oracle_to_state, rel,
                            lam_rel_operands, rel_list, rounded_inputs, state_to_oracle, u_elem_err, u_weights)
from tests.oracle_problems import oracle_problem, tiny_spec

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)


# ---------------------------------------------------------------------------
# prox (eq. Prox_sol)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("eps,lam", [(0.5, 0.1), (0.5, 1.0), (0.5, 2.0), (0.1, 20.0), (0.9, 0.5), (0.9, 5.0)])
def test_prox_parity(eps, lam):
    say("prox", eps, lam)
    rng = np.random.default_rng(int(100 * eps + lam))
    n = 200_003                                    # ragged length
    y = (rng.standard_normal(n) + 1j * rng.standard_normal(n)) * rng.uniform(0, 3, n)
    sf = np.abs(rng.standard_normal(n)) * 2
    y[:100] = 0                                    # tie rule sign(0) = +1
    sf[100:200] = 0                                # f = 0
    y32 = y.astype(np.complex64)
    sf32 = sf.astype(np.float32)
    z = host(odp.prox_stagm(dev_c64(y32), dev_f32(sf32), eps, lam))
    want = stagm.prox(y32.astype(np.complex128), sf32.astype(np.float64) ** 2, eps, lam)
    err = np.abs(z - want)
    scale = np.abs(want) + sf32 + np.abs(y32)
    assert np.all(err <= 2e-6 * scale + 1e-30), float((err / (scale + 1e-30)).max())
    assert np.all(z[:100].imag == 0) and np.all(z[:100].real >= 0)
    if eps - (1 - eps) / lam > 0:
        assert np.any(np.abs(y32) < (eps - (1 - eps) / lam) * sf32)   # truncated branch exercised


def test_prox_in_place_and_empty():
    y = dev_c64(np.array([1 + 1j, 0, -2j], np.complex64))
    sf = dev_f32(np.array([1.0, 2.0, 0.5], np.float32))
    want = stagm.prox(host(y), host(sf) ** 2, 0.5, 0.3)
    odp.prox_stagm(y, sf, 0.5, 0.3, out=y)
    np.testing.assert_allclose(host(y), want, rtol=1e-6, atol=1e-7)
    e = torch.empty(0, dtype=torch.complex64, device="cuda")
    odp.prox_stagm(e, torch.empty(0, dtype=torch.float32, device="cuda"), 0.5, 0.3)


# ---------------------------------------------------------------------------
# A, A*, A*A (Sec. 2, eq. AtA) for every supported frame size
# ---------------------------------------------------------------------------

OPS_CASES = [  # (n, p, step, jitter, dy, dx)
    (96, 32, 8, 1, 1, 2),
    (200, 64, 12, 2, 2, 2),
    (320, 128, 24, 3, 1, 2),
]


@pytest.mark.parametrize("case", OPS_CASES, ids=lambda c: f"p{c[1]}")
def test_forward_adjoint_parity(case):
    n, p, step, jit, dy, dx = case
    say("operators", case)
    rng = np.random.default_rng(p)
    off, grid = synthetic.raster_offsets(n, p, step, jit, rng)
    sub = synthetic.block_partition(grid, dy, dx)
    w = (synthetic.make_probe(p, p * 0.38, 0.02) + 0.02 * (rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p))))
    w = w.astype(np.complex64).astype(np.complex128)
    u = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))).astype(np.complex64).astype(np.complex128)
    y = (rng.standard_normal((len(off), p, p)) + 1j * rng.standard_normal((len(off), p, p))).astype(np.complex64).astype(np.complex128)
    plan = odp.Plan(n, n, p, off, sub, r=1.0)
    plan.bind(dev_f32(np.ones((len(off), p, p))), dev_c64(w))
    X = host(plan.forward(dev_c64(u), dev_c64(w)))
    Xo = ops.forward(u, w, off)
    per_frame = np.linalg.norm((X - Xo).reshape(len(off), -1), axis=1) / np.linalg.norm(Xo.reshape(len(off), -1), axis=1)
    assert per_frame.max() <= 1e-5, per_frame.max()
    Ay = host(plan.adjoint(dev_c64(y), dev_c64(w)))
    Ayo = ops.adjoint(y, w, off, (n, n))
    assert rel(Ay, Ayo) <= 1e-5
    # adjoint identity on the GPU's own results
    lhs, rhs = np.vdot(X, y), np.vdot(u, Ay)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    # A*A u = diag(sum_j S_j^T |w|^2) u
    AtAu = host(plan.adjoint(plan.forward(dev_c64(u), dev_c64(w)), dev_c64(w)))
    assert rel(AtAu, ops.illumination(w, off, (n, n)) * u) <= 1e-5


def test_forward_single_frame():
    say("forward single frame")
    p = 64
    rng = np.random.default_rng(1)
    off = np.array([[3, 5]], np.int32)
    w = synthetic.make_probe(p, 24, 0.02).astype(np.complex64).astype(np.complex128)
    u = (rng.standard_normal((70, 72)) + 1j * rng.standard_normal((70, 72))).astype(np.complex64).astype(np.complex128)
    plan = odp.Plan(70, 72, p, off, np.zeros(1, np.int32))
    plan.bind(dev_f32(np.ones((1, p, p))), dev_c64(w))
    X = host(plan.forward(dev_c64(u), dev_c64(w)))
    assert rel(X, ops.forward(u, w, off)) <= 1e-5


# ---------------------------------------------------------------------------
# one ADMM iteration (Alg. 2) from an arbitrary state
# ---------------------------------------------------------------------------

STEP_CASES = [
    ("c1_shape", tiny_spec(n=128, p=32, step=8, jitter=1, dy=1, dx=2, radius=12), 0.1),
    ("grid3x3_eta2", tiny_spec(n=160, p=32, step=8, jitter=2, dy=3, dx=3, radius=12, peak=1e4), 2.0),
    ("grid2x3_p64", tiny_spec(n=256, p=64, step=16, jitter=2, dy=2, dx=3, radius=24, peak=1e3), 0.1),
    ("narrow_blocks", tiny_spec(n=120, p=32, step=6, jitter=1, dy=2, dx=5, radius=12), 0.5),
    ("grid2x2_p128", tiny_spec(n=256, p=128, step=32, jitter=2, dy=2, dx=2, radius=48, peak=1e3), 0.1),
]


@pytest.mark.parametrize("name,spec,eta", STEP_CASES, ids=lambda c: c if isinstance(c, str) else "")
def test_one_iteration_from_random_state(name, spec, eta):
    say("one iteration", name)
    P = oracle_problem(spec, eta=eta)
    g = P["geom"]
    w, _, f = rounded_inputs(P)
    plan = gpu_plan(P)
    st = plan.new_state()
    rng = np.random.default_rng(7)
    ost = init_state(g)
    ost.u = [(1 + 0.3 * (rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape))).astype(np.complex64).astype(np.complex128) for a in ost.u]
    ost.gamma = (0.05 * (rng.standard_normal(ost.gamma.shape) + 1j * rng.standard_normal(ost.gamma.shape))).astype(np.complex64).astype(np.complex128)
    ost.lam = {k: (0.1 * (rng.standard_normal(v.shape) + 1j * rng.standard_normal(v.shape))).astype(np.complex64).astype(np.complex128) for k, v in ost.lam.items()}
    oracle_to_state(ost, st)
    stats = plan.iterate(st, 1, stats=True)
    new, ostats = od2pm_step(g, w, f, ost, P["eps"], eta, P["r"])
    got = state_to_oracle(st)
    e = dict(u=rel_list(got.u, new.u), gamma=rel(got.gamma, new.gamma),
             lam=max(rel(got.lam[k], new.lam[k]) for k in new.lam))
    assert max(e.values()) <= 1e-5, e
    el = _elementwise(P, g, w, f, eta, got, new)
    say("element-wise", el)
    assert max(el.values()) <= 1e-5, el
    s = host(stats)[0]
    assert abs(s[0] - ostats["RF"]) <= 1e-5 * ostats["RF"]
    assert abs(s[1] - ostats["RE"]) <= 1e-4 * ostats["RE"]
    assert abs(s[2] - ostats["G"]) <= 1e-5 * ostats["G"]


def _elementwise(P, g, w, f, eta, got, new):
    """Element-wise errors of the iterate produced by the last iteration: u through its
    closed form's numerator, Gamma at the scale of y = Gamma^n + A u^n (= Gamma^{n+1} +
    z^{n+1}) with the prox's conditioning, Lam at the scale of its operands."""
    y = new.gamma + new.z
    return dict(u=u_elem_err(got.u, new.u, u_weights(g, lambda d: w, eta, P["r"])),
                gamma=gamma_elem_err(got.gamma, new.gamma, y, np.sqrt(f), P["eps"], eta),
                lam=lam_elem_err(got.lam, new.lam, new.u, g) if new.lam else 0.0)


def _interleaved(P, D, eta):
    """Frame j goes to subdomain j mod D: every subdomain spans the image, so a pixel
    lies in up to D subdomains (D = 3 leaves an idle copy group of four, D > 4 takes
    the path for five to sixteen copies)."""
    pr = P["pr"]
    spec = pr["spec"]
    pr["frame_sub"] = (np.arange(len(pr["offsets"])) % D).astype(np.int32)
    g = build_geometry(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"])
    P["geom"] = g
    P["den"] = [subdomain_illumination(g, pr["w"], d) for d in range(g.D)]
    P["r"] = 0.5 * eta * max(float(a.max()) for a in P["den"])
    return P


@pytest.mark.parametrize("D", [3, 5, 8, 12, 16])
def test_one_iteration_many_copies(D):
    say("one iteration, interleaved subdomains", D)
    eta = 0.3
    P = _interleaved(oracle_problem(tiny_spec(n=96, p=32, step=8, jitter=1, radius=12, peak=1e4), eta=eta), D, eta)
    g = P["geom"]
    w, _, f = rounded_inputs(P)
    plan = gpu_plan(P)
    assert plan.info.max_cover == D
    st = plan.new_state()
    rng = np.random.default_rng(D)
    ost = init_state(g)
    ost.u = [(1 + 0.3 * (rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape))).astype(np.complex64).astype(np.complex128) for a in ost.u]
    ost.lam = {k: (0.1 * (rng.standard_normal(v.shape) + 1j * rng.standard_normal(v.shape))).astype(np.complex64).astype(np.complex128) for k, v in ost.lam.items()}
    oracle_to_state(ost, st)
    stats = host(plan.iterate(st, 2, stats=True))
    mid, h1 = od2pm_run(g, w, f, P["eps"], eta, P["r"], 1, state=ost)
    new, h2 = od2pm_step(g, w, f, mid, P["eps"], eta, P["r"])     # keeps z for the element bounds
    h = h1 + [h2]
    got = state_to_oracle(st)
    e = dict(u=rel_list(got.u, new.u), gamma=rel(got.gamma, new.gamma),
             lam=max(rel(got.lam[k], new.lam[k]) for k in new.lam))
    assert max(e.values()) <= 1e-5, e
    el = _elementwise(P, g, w, f, eta, got, new)
    say("element-wise", el)
    assert max(el.values()) <= 1e-5, el
    np.testing.assert_allclose(stats[:, 1], [x["RE"] for x in h], rtol=1e-4)


# ---------------------------------------------------------------------------
# whole runs from Step 0
# ---------------------------------------------------------------------------

def test_c1_full_run_parity():
    spec = synthetic.CONFIGS["c1"]
    say("c1 full", spec.iters)
    P = oracle_problem(spec)
    g = P["geom"]
    w, _, f = rounded_inputs(P)
    plan = gpu_plan(P)
    st = plan.new_state()
    stats = host(plan.iterate(st, spec.iters, stats=True))
    ost, hist = od2pm_run(g, w, f, P["eps"], P["eta"], P["r"], spec.iters)
    got = state_to_oracle(st)
    assert rel_list(got.u, ost.u) <= 1e-3
    u_gpu = host(plan.merge(st))
    assert rel(u_gpu, merge(g, ost.u)) <= 1e-3
    rf = np.array([h["RF"] for h in hist])
    np.testing.assert_allclose(stats[:, 0], rf, rtol=1e-3)
    assert stats[-1, 0] < 0.01 * stats[0, 0]        # it converges


def test_c2_full_size_iterations():
    spec = synthetic.CONFIGS["c2"]
    say("c2 full size, 3 iterations")
    P = oracle_problem(spec)
    g = P["geom"]
    w, _, f = rounded_inputs(P)
    plan = gpu_plan(P)
    st = plan.new_state()
    stats = host(plan.iterate(st, 3, stats=True))
    ost, hist = od2pm_run(g, w, f, P["eps"], P["eta"], P["r"], 3)
    got = state_to_oracle(st)
    assert rel_list(got.u, ost.u) <= 1e-5
    assert rel(got.gamma, ost.gamma) <= 1e-5
    say("Lam plain relative", max(rel(got.lam[k], ost.lam[k]) for k in ost.lam))
    assert lam_rel_operands(got.lam, ost.lam, ost.u, g) <= 1e-5
    np.testing.assert_allclose(stats[:, 0], [h["RF"] for h in hist], rtol=1e-5)
    np.testing.assert_allclose(stats[:, 2], [h["G"] for h in hist], rtol=1e-5)


def test_p128_single_domain_run():
    spec = tiny_spec(n=256, p=128, step=32, jitter=0, dy=1, dx=1, radius=48, peak=None)
    say("p128 D=1 run")
    P = oracle_problem(spec)
    w, _, f = rounded_inputs(P)
    plan = gpu_plan(P)
    st = plan.new_state()
    plan.iterate(st, 10)
    ost, _ = od2pm_run(P["geom"], w, f, P["eps"], P["eta"], P["r"], 10)
    assert rel_list(state_to_oracle(st).u, ost.u) <= 1e-4


def test_resume_matches_uninterrupted():
    spec = synthetic.CONFIGS["c1"]
    say("resume")
    P = oracle_problem(spec)
    plan = gpu_plan(P)
    a = plan.new_state()
    plan.iterate(a, 6)
    b = plan.new_state()
    plan.iterate(b, 2)
    c = b.clone()                      # checkpoint = a copy of the state buffer
    plan.iterate(c, 4)
    # every reduction runs in a fixed order: resuming from a copy is bit for bit
    from tests.gpu_util import same_state
    assert same_state(a, c)


def test_held_pixels_stay_one():
    # a probe that leaves the window corners dark: uncovered corner pixels are never illuminated
    spec = tiny_spec(n=64, p=32, step=16, jitter=0, dy=1, dx=1, radius=10)
    say("held pixels")
    P = oracle_problem(spec)
    plan = gpu_plan(P)
    st = plan.new_state()
    plan.iterate(st, 3)
    den = subdomain_illumination(P["geom"], P["pr"]["w"], 0)
    u = host(st.u_sub()[0])
    assert np.any(den == 0)
    assert np.all(u[den == 0] == 1.0)


def test_zero_iterations_leave_the_state_and_negative_counts_are_refused():
    from paper_2011_00162_amd._lib import ODP_EINVAL
    from tests.gpu_util import same_state
    spec = tiny_spec(n=128, p=32, step=8, jitter=1, dy=2, dx=2, radius=12, peak=1e4)
    say("zero iterations")
    P = oracle_problem(spec)
    plan = gpu_plan(P)
    a, b = plan.new_state(), plan.new_state()
    plan.iterate(a, 1)
    c = a.clone()
    assert plan.iterate(a, 0, stats=True) is None
    assert same_state(a, c) and not same_state(a, b)
    with pytest.raises(odp.OdpError) as e:
        plan.iterate(a, -1)
    assert e.value.code == ODP_EINVAL
    assert same_state(a, c)

"""GPU parity of the amplitude loss and its hand-written backward (dL/du, dL/dw)
against the FP64 oracle, whose gradient is pinned by finite differences."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import synthetic
import paper_2011_00162_amd as odp
from oracle import amploss, operators as ops
from tests.gpu_util import dev_c64, dev_f32, host, rel

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)


def _case(n, dy=1, dx=1, seed=3):
    spec = synthetic.crop_spec(synthetic.CONFIGS["c3"], n, dy=dy, dx=dx)
    pr = synthetic.draw_problem(spec)
    w = pr["w"].astype(np.complex64).astype(np.complex128)
    f = ops.intensities(pr["u_true"], w, pr["offsets"])
    sf32 = np.sqrt(f).astype(np.float32)
    f = sf32.astype(np.float64) ** 2
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    u = (pr["u_true"] * (1 + 0.1 * xi)).astype(np.complex64).astype(np.complex128)
    plan = odp.Plan(n, n, spec.p, pr["offsets"], pr["frame_sub"], r=1.0)
    plan.bind(dev_f32(sf32), dev_c64(w))
    return plan, u, w, f, pr["offsets"]


@pytest.mark.parametrize("n,dy,dx", [(256, 1, 1), (256, 2, 2), (1024, 1, 1)], ids=["crop256", "crop256_2x2", "c3_full"])
def test_loss_and_gradients(n, dy, dx):
    say("amplitude loss", n, dy, dx)
    plan, u, w, f, off = _case(n, dy, dx)
    for uu in (u, np.ones_like(u)):
        loss, gu, gw = plan.amp_loss(dev_c64(uu), dev_c64(w))
        L, gu_o, gw_o = amploss.grad(uu, w, off, f)
        assert abs(host(loss)[0] - L) <= 1e-5 * L
        assert rel(host(gu), gu_o) <= 1e-5, rel(host(gu), gu_o)
        assert rel(host(gw), gw_o) <= 1e-5, rel(host(gw), gw_o)


@pytest.mark.parametrize("want_u,want_w", [(True, False), (False, True), (False, False)],
                         ids=["grad_u_only", "grad_w_only", "loss_only"])
def test_one_gradient_or_none(want_u, want_w):
    # the loss total is formed by a different kernel depending on which gradients are
    # asked for; every combination gives the oracle's loss and requested gradients
    say("amplitude loss, gradients", want_u, want_w)
    plan, u, w, f, off = _case(256, 2, 2)
    loss, gu, gw = plan.amp_loss(dev_c64(u), dev_c64(w), grad_u=want_u, grad_w=want_w)
    L, gu_o, gw_o = amploss.grad(u, w, off, f)
    assert abs(host(loss)[0] - L) <= 1e-5 * L
    assert (gu is None) != want_u and (gw is None) != want_w
    if want_u:
        assert rel(host(gu), gu_o) <= 1e-5, rel(host(gu), gu_o)
    if want_w:
        assert rel(host(gw), gw_o) <= 1e-5, rel(host(gw), gw_o)


def test_autograd_function_matches_entry_point():
    say("autograd")
    plan, u, w, f, off = _case(256)
    ut = dev_c64(u).requires_grad_(True)
    wt = dev_c64(w).requires_grad_(True)
    L = odp.amplitude_loss(ut, wt, plan)
    (3.0 * L).backward()
    _, gu_o, gw_o = amploss.grad(u, w, off, f)
    assert rel(host(ut.grad), 3.0 * gu_o) <= 1e-5
    assert rel(host(wt.grad), 3.0 * gw_o) <= 1e-5


def test_gradient_at_truth_vanishes():
    say("gradient at the truth")
    spec = synthetic.crop_spec(synthetic.CONFIGS["c3"], 256)
    pr = synthetic.draw_problem(spec)
    u = pr["u_true"].astype(np.complex64)
    w = pr["w"].astype(np.complex64)
    plan = odp.Plan(256, 256, 128, pr["offsets"], pr["frame_sub"], r=1.0)
    X = plan.bind(torch.ones((25, 128, 128), device="cuda"), dev_c64(w)).forward(dev_c64(u), dev_c64(w))
    sf = X.abs().float().contiguous()
    plan2 = odp.Plan(256, 256, 128, pr["offsets"], pr["frame_sub"], r=1.0)
    plan2.bind(sf, dev_c64(w))
    loss, gu, gw = plan2.amp_loss(dev_c64(u), dev_c64(w))
    assert host(loss)[0] < 1e-9 * float((sf.double() ** 2).sum())
    assert float(gu.abs().max()) < 1e-4 and float(gw.abs().max()) < 1e-3


def test_gradient_is_zero_where_no_frame_reaches():
    """A 300 x 300 image scanned only over its top-left 256 x 256: the pixels no window
    reaches get dL/du = 0 (the library clears what its tiles do not cover)."""
    say("amplitude loss, uncovered border")
    n, p = 300, 128
    off, grid = synthetic.raster_offsets(256, p, 32, 0, None)
    sub = synthetic.block_partition(grid, 1, 1)
    rng = np.random.default_rng(4)
    u = ((1 + 0.2 * rng.standard_normal((n, n))) * np.exp(0.3j * rng.standard_normal((n, n)))).astype(
        np.complex64).astype(np.complex128)
    w = synthetic.make_probe(p, 48.0, 0.01).astype(np.complex64).astype(np.complex128)
    f = ops.intensities(u * (1 + 0.05 * rng.standard_normal((n, n))), w, off)
    sf32 = np.sqrt(f).astype(np.float32)
    f = sf32.astype(np.float64) ** 2
    plan = odp.Plan(n, n, p, off, sub, r=1.0)
    plan.bind(dev_f32(sf32), dev_c64(w))
    loss, gu, gw = plan.amp_loss(dev_c64(u), dev_c64(w))
    L, gu_o, gw_o = amploss.grad(u, w, off, f)
    gu = host(gu)
    assert np.all(gu[256:, :] == 0) and np.all(gu[:, 256:] == 0)
    assert rel(gu, gu_o) <= 1e-5 and rel(host(gw), gw_o) <= 1e-5
    assert abs(host(loss)[0] - L) <= 1e-5 * L

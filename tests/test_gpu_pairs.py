"""The paired pixel pull gives the same iterates bit for bit as the one-pixel pull.

Where every frame window of a tile starts at a column of the tile's parity (even raster
offsets), a thread of the pixel update holds two row neighbours and fetches both from a
frame with one 16-byte load (odp_plan_set_pixel_pairs, on by default).  Each pixel's sum
still runs over the same frames in the same order, so u, Lam, Gamma and (blind) the probe
copies must match the one-pixel pull exactly; the FP64 statistics add the pixels in
another order and agree to rounding.  The oracle parity tests cover the one-pixel pull
on jittered scans; the full-size tests run the paired one against the oracle."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_2011_00162_amd as odp
from tests.gpu_util import dev_c64, gpu_plan, host
from tests.oracle_problems import oracle_problem, tiny_spec
from tests.test_gpu_streaming import _parts, _start

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)


# unjittered scans: every window column even, so every tiling pairs its pixels
CASES = [
    ("p32_fft", tiny_spec(n=128, p=32, step=8, jitter=0, dy=2, dx=2, radius=12, peak=1e4), odp.ODP_FFT_F32),
    ("p64_fft", tiny_spec(n=256, p=64, step=16, jitter=0, dy=2, dx=3, radius=24, peak=1e3), odp.ODP_FFT_F32),
    ("p128_fft", tiny_spec(n=256, p=128, step=32, jitter=0, dy=2, dx=2, radius=48, peak=1e3), odp.ODP_FFT_F32),
    ("p128_hybrid", tiny_spec(n=256, p=128, step=32, jitter=0, dy=2, dx=2, radius=48, peak=1e3), odp.ODP_HYBRID_MFMA),
]


@pytest.mark.parametrize("tiling", [0, 1, 2])
@pytest.mark.parametrize("blind", [False, True], ids=["known_probe", "blind"])
@pytest.mark.parametrize("name,spec,transform", CASES, ids=lambda c: c if isinstance(c, str) else "")
def test_paired_pull_is_bit_identical(name, spec, transform, blind, tiling):
    say("pixel pairs on/off", name, "blind" if blind else "known probe", "tiling", tiling)
    P = oracle_problem(spec)
    mu = 0.5 * P["eta"] * max(len(fr) for fr in P["geom"].frames_of) if blind else 0.0
    runs = []
    for mode in (0, 1):
        plan = gpu_plan(P, blind=blind, mu=mu)
        plan.set_tuning(transform, 1, tiling)
        plan.set_pixel_pairs(mode)
        assert plan.tuning().pixel_pairs == mode
        st = _start(plan, P, blind)
        plan.iterate(st, 3)                      # the timed path (no statistics)
        stats = host(plan.iterate(st, 2, stats=True))   # the statistics variants
        torch.cuda.synchronize()
        runs.append((_parts(plan, st), stats))
    (a0, s0), (a1, s1) = runs
    differ = {k: int((a0[k] != a1[k]).sum()) for k in a0 if not torch.equal(a0[k], a1[k])}
    assert not differ, differ
    np.testing.assert_allclose(s1, s0, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("dy", [1, 2])
def test_paired_pull_gives_the_same_loss_gradient(dy):
    """The amplitude loss's image gradient pulls the same way: bit-identical dL/du with the
    paired and the one-pixel pull (256^2 crops of the loss workload, one and 2 x 2
    subdomains, every tiling)."""
    from tests.test_gpu_loss import _case
    say("loss gradient, pixel pairs on/off, subdomains", dy, "x", dy)
    plan, u, w, f, off = _case(256, dy, dy)
    L = odp.lib()
    for tiling in (0, 1, 2):
        assert L.odp_plan_set_tuning(plan._h, odp.ODP_FFT_F32, 1, tiling, None) == 0
        out = []
        for mode in (0, 1):
            plan.set_pixel_pairs(mode)
            assert plan.tuning().pixel_pairs == mode
            loss, gu, gw = plan.amp_loss(dev_c64(u), dev_c64(w))
            torch.cuda.synchronize()
            out.append((host(loss), gu.clone(), gw.clone()))
        (l0, u0, w0), (l1, u1, w1) = out
        assert torch.equal(u0, u1), (tiling, int((u0 != u1).sum()))
        assert torch.equal(w0, w1) and np.array_equal(l0, l1)

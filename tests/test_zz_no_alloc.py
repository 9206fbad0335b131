"""The allocation-free initial probe (odp_blind_initial_probe_static) against the
plan-based entry point (odp_blind_initial_probe) and the FP64 oracle: two calls in a
row on one device, the second with fewer frames and a smaller probe, so the second
reads a static scratch that still holds the first call's partial sums."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import paper_2011_00162_amd as odp
from oracle import blind
from paper_2011_00162_amd._lib import ODP_EINVAL, ODP_ENOMEM, ODP_EUNSUPPORTED
from tests.gpu_util import dev_f32, gpu_plan, host, rel, rounded_inputs
from tests.oracle_problems import oracle_problem, tiny_spec

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)


def _case(n, p, step, rad, peak):
    spec = tiny_spec(n=n, p=p, step=step, jitter=2, dy=2, dx=2, radius=rad, peak=peak)
    P = oracle_problem(spec)
    _, sf32, _ = rounded_inputs(P)
    return P, sf32


def test_static_initial_probe_matches_plan_entry_point():
    # first call: p = 128, 49 frames (more than the 32 chunks: two frames per chunk);
    # second call: p = 64, 25 frames (one frame per chunk), on the scratch the first left
    for n, p, step, rad, peak in ((320, 128, 32, 48, 1e4), (192, 64, 32, 24, 1e3)):
        say("static initial probe", p)
        P, sf32 = _case(n, p, step, rad, peak)
        J = sf32.shape[0]
        plan = gpu_plan(P, blind=True, mu=1.0)
        want_plan = host(plan.blind_initial_probe())
        torch.cuda.synchronize()
        got = host(odp.blind_initial_probe_static(dev_f32(sf32)))
        want = blind.initial_probe(sf32.astype(np.float64))
        say("J", J, "vs plan", rel(got, want_plan), "vs oracle", rel(got, want))
        assert rel(got, want_plan) <= 1e-5
        assert rel(got, want) <= 1e-5


def test_static_initial_probe_refuses_sizes():
    sf = torch.zeros((2, 256, 256), dtype=torch.float32, device="cuda")
    with pytest.raises(odp.OdpError) as e:
        odp.blind_initial_probe_static(sf)
    assert e.value.code == ODP_ENOMEM and "static scratch" in str(e.value)
    with pytest.raises(odp.OdpError) as e:
        odp.blind_initial_probe_static(torch.zeros((2, 48, 48), dtype=torch.float32, device="cuda"))
    assert e.value.code == ODP_EUNSUPPORTED
    with pytest.raises(odp.OdpError) as e:
        odp.blind_initial_probe_static(torch.zeros((0, 32, 32), dtype=torch.float32, device="cuda"))
    assert e.value.code == ODP_EINVAL

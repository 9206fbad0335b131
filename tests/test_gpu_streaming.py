"""The streaming (non-temporal) kernel variants give bit-identical results.

A plan accesses its frame arrays with non-temporal loads and stores when they exceed the
Infinity Cache (odp_plan_set_streaming, mode -1).  That changes cache policy only, not the
arithmetic or its order, so on the same inputs the streaming and the ordinary variants of
every sweep, probe-copy and pixel kernel must produce the same state bit for bit.  The
ordinary variants are checked against the FP64 oracle elsewhere; these small problems force
each mode so that the streaming variants of every transform are exercised (at full size
they are what runs)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import synthetic
import paper_2011_00162_amd as odp
from tests.gpu_util import dev_c64, gpu_plan, host, rounded_inputs
from tests.oracle_problems import oracle_problem, tiny_spec

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)


CASES = [
    ("p32_fft", tiny_spec(n=128, p=32, step=8, jitter=1, dy=2, dx=2, radius=12, peak=1e4), odp.ODP_FFT_F32),
    ("p64_fft", tiny_spec(n=256, p=64, step=16, jitter=2, dy=2, dx=3, radius=24, peak=1e3), odp.ODP_FFT_F32),
    ("p64_dft", tiny_spec(n=256, p=64, step=16, jitter=2, dy=2, dx=3, radius=24, peak=1e3), odp.ODP_DFT_SPLIT_BF16),
    ("p64_hybrid", tiny_spec(n=256, p=64, step=16, jitter=2, dy=2, dx=3, radius=24, peak=1e3), odp.ODP_HYBRID_MFMA),
    ("p128_fft", tiny_spec(n=256, p=128, step=32, jitter=2, dy=2, dx=2, radius=48, peak=1e3), odp.ODP_FFT_F32),
    ("p128_hybrid", tiny_spec(n=256, p=128, step=32, jitter=2, dy=2, dx=2, radius=48, peak=1e3), odp.ODP_HYBRID_MFMA),
]


def _start(plan, P, blind):
    if not blind:
        return plan.new_state()
    _, _, f = rounded_inputs(P)
    p = P["pr"]["spec"].p
    w0 = synthetic.make_probe(p, P["pr"]["spec"].radius * 0.85, 0.0)
    w0 = w0 * np.sqrt(f.sum(axis=(1, 2)).mean() / max(np.sum(np.abs(w0) ** 2), 1e-30))
    return plan.new_state(w0=dev_c64(w0.astype(np.complex64).astype(np.complex128)))


def _parts(plan, st):
    """The state's defined arrays (the buffer's alignment padding is never written)."""
    out = {"u": torch.cat([t.reshape(-1) for t in st.u_sub()]), "gamma": st.gamma().reshape(-1)}
    lam = st.lam()
    if lam:
        out["lam"] = torch.cat([v.reshape(-1) for v in lam.values()])
    if plan.blind:
        out.update(w=st.probe().reshape(-1), w_sub=st.probe_copies().reshape(-1),
                   delta=st.probe_multipliers().reshape(-1))
    return {k: v.clone() for k, v in out.items()}


@pytest.mark.parametrize("blind", [False, True], ids=["known_probe", "blind"])
@pytest.mark.parametrize("name,spec,transform", CASES, ids=lambda c: c if isinstance(c, str) else "")
def test_streaming_variants_are_bit_identical(name, spec, transform, blind):
    say("streaming on/off", name, "blind" if blind else "known probe")
    P = oracle_problem(spec)
    mu = 0.5 * P["eta"] * max(len(fr) for fr in P["geom"].frames_of) if blind else 0.0
    runs = []
    for mode in (0, 1):
        plan = gpu_plan(P, blind=blind, mu=mu)
        plan.set_tuning(transform, 1, 0)
        plan.set_streaming(mode)
        st = _start(plan, P, blind)
        plan.iterate(st, 3)                      # the timed path (no statistics)
        stats = host(plan.iterate(st, 2, stats=True))   # the statistics variants
        torch.cuda.synchronize()
        runs.append((_parts(plan, st), stats))
    (a0, s0), (a1, s1) = runs
    differ = {k: int((a0[k] != a1[k]).sum()) for k in a0 if not torch.equal(a0[k], a1[k])}
    assert not differ, differ
    assert np.array_equal(s0, s1), (s0, s1)


def test_streaming_mode_is_validated():
    P = oracle_problem(CASES[0][1])
    plan = gpu_plan(P)
    for mode in (-1, 0, 1):
        plan.set_streaming(mode)
    with pytest.raises(Exception):
        plan.set_streaming(2)

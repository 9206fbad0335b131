"""Helpers for the GPU parity tests: build a bound plan from an oracle problem and
move states between the device layout and the oracle's representation.

Both sides start from the same FP32-rounded inputs: the oracle receives the
probe rounded to complex64 and intensities whose square roots are the float32
values the GPU reads, so the comparison isolates the arithmetic.
"""
from __future__ import annotations

import numpy as np
import torch

import paper_2011_00162_amd as odp
from oracle.od2p import OD2PState

DEV = "cuda"


def dev_c64(x) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.complex64))).to(DEV)


def dev_f32(x) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float32))).to(DEV)


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


def rounded_inputs(P):
    """(w as complex64-rounded complex128, sqrt_f float32, f = sqrt_f^2 in float64)."""
    w = np.asarray(P["pr"]["w"], dtype=np.complex64).astype(np.complex128)
    sf32 = np.sqrt(P["f"]).astype(np.float32)
    return w, sf32, sf32.astype(np.float64) ** 2


def gpu_plan(P, eta=None, r=None, eps=None, blind=False, mu=0.0, gamma=0.0, mask=None, w=None):
    spec = P["pr"]["spec"]
    w_r, sf32, _ = rounded_inputs(P)
    plan = odp.Plan(spec.n, spec.n, spec.p, P["pr"]["offsets"], P["pr"]["frame_sub"],
                    eps=P["eps"] if eps is None else eps, eta=P["eta"] if eta is None else eta,
                    r=P["r"] if r is None else r, mu=mu, gamma=gamma, blind=blind, probe_fmask=mask)
    plan.bind(dev_f32(sf32), dev_c64(w_r if w is None else w))
    return plan


def state_to_oracle(state: "odp.State") -> OD2PState:
    torch.cuda.synchronize()
    u = [host(t) for t in state.u_sub()]
    lam = {k: host(v) for k, v in state.lam().items()}
    return OD2PState(u=u, gamma=host(state.gamma()), lam=lam)


def oracle_to_state(ost: OD2PState, state: "odp.State") -> None:
    for dst, src in zip(state.u_sub(), ost.u):
        dst.copy_(torch.from_numpy(src.astype(np.complex64)))
    state.gamma().copy_(torch.from_numpy(ost.gamma.astype(np.complex64)))
    lam = state.lam()
    for k, v in ost.lam.items():
        lam[k].copy_(torch.from_numpy(v.astype(np.complex64)))
    torch.cuda.synchronize()


def rel(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rel_list(a: list, b: list) -> float:
    return max(rel(x, y) for x, y in zip(a, b))


def same_state(a: "odp.State", b: "odp.State") -> bool:
    """Bit-for-bit equality of the state variables (u_d, Gamma, Lam and, when blind,
    w, w_d, Delta); the alignment gaps between them carry no data."""
    torch.cuda.synchronize()
    if not all(torch.equal(x, y) for x, y in zip(a.u_sub(), b.u_sub())):
        return False
    if not torch.equal(a.gamma(), b.gamma()):
        return False
    la, lb = a.lam(), b.lam()
    if not all(torch.equal(la[k], lb[k]) for k in la):
        return False
    if a.plan.blind:
        return (torch.equal(a.probe(), b.probe()) and torch.equal(a.probe_copies(), b.probe_copies())
                and torch.equal(a.probe_multipliers(), b.probe_multipliers()))
    return True

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


# ---------------------------------------------------------------------------
# element-wise bounds (a norm over a whole stack can hide an error confined to dark
# pixels or weak frequencies).  Each quantity is compared at the scale of the operands
# its FP32 arithmetic combines, plus an absolute floor: 1e-3 of that scale's maximum for
# pixel-domain sums, and the rms of the array for values that come straight out of a
# transform (an FP32 FFT's error in one output is absolute, a share of the frame's norm:
# a norm-relative bound tol allows tol * rms per element).
# ---------------------------------------------------------------------------

FLOOR = 1e-3


def elem_err(a, b, scale, floor="max") -> float:
    """max_k |a_k - b_k| / (scale_k + floor), floor = FLOOR * max scale or rms(scale)."""
    a, b, scale = np.asarray(a), np.asarray(b), np.asarray(scale, dtype=np.float64)
    fl = FLOOR * scale.max() if floor == "max" else float(np.sqrt(np.mean(scale ** 2)))
    s = scale + fl
    s = np.where(s > 0, s, 1.0)
    return float((np.abs(a - b) / s).max())


def u_weights(g, w_of_sub, eta, r, gamma=0.0) -> list:
    """The u-step denominator eta*den_d + r*k_d + gamma per subdomain pixel (eqs.
    Alg1-solver-u, blind_U): u_k is its numerator divided by it, so the FP32 error of u_k
    is the numerator's error over this weight.  w_of_sub(d) is the probe subdomain d uses."""
    from oracle.geometry import multiplicity
    from oracle.od2p import subdomain_illumination
    return [eta * subdomain_illumination(g, w_of_sub(d), d) + r * multiplicity(g, d) + gamma
            for d in range(g.D)]


def u_elem_err(got: list, want: list, weights: list, floor="max") -> float:
    """Element-wise error of u through its closed form's numerator (weight * u).  The
    numerator is a pull of inverse transforms: the FP32 paths meet the stricter 1e-3 * max
    floor; split-BF16 transforms (error about 2^-17 of the frame's rms per element) take
    the rms floor."""
    return max(elem_err(wt * a, wt * b, np.abs(wt * b), floor) for a, b, wt in zip(got, want, weights))


def u_weighted_rel(got: list, want: list, den: list) -> float:
    """||A_d (u_gpu - u_or)|| / ||A_d u_or|| over all subdomains, with ||A_d x||^2 =
    sum den_d |x|^2 (F unitary, diag(A_d* A_d) = den_d, eq. AtA)."""
    num = sum(float(np.sum(dd * np.abs(a - b) ** 2)) for a, b, dd in zip(got, want, den))
    ref = sum(float(np.sum(dd * np.abs(b) ** 2)) for b, dd in zip(want, den))
    return float(np.sqrt(num / ref))


def lam_elem_err(got: dict, want: dict, u_new: list, g) -> float:
    """Lam^{n+1} = Lam^n + pi u^{n+1} - v^{n+1} (eq. updateM-2-multi) at the scale of its
    operands |Lam^{n+1}| + |pi u^{n+1}|."""
    worst = 0.0
    for (i1, i2, rc) in g.pairs:
        for a, b in ((i1, i2), (i2, i1)):
            pu = u_new[a][g.restrict(a, rc)]
            worst = max(worst, elem_err(got[(a, b)], want[(a, b)], np.abs(want[(a, b)]) + np.abs(pu)))
    return worst


def gamma_elem_err(got, want, y, sqrt_f, eps, lam) -> float:
    """Gamma^{n+1} = y - Prox(y) (eqs. updateM-1, Prox_sol) per frame, at the scale of the
    transform that produced y, |y_k| + rms(y_j) (the per-frame operator bound, relative in
    norm, allows the frame's rms per element), times the map's local Lipschitz bound:
    (1 + sqrt(f_k)/|y_k|)/(1 + lam) on the AGM branch (its angular part divides by |y|),
    c/(lam - c) on the truncated branch (c = (1 - eps)/eps), and 1.  Where y_k = 0 the
    phase of Gamma_k is a tie (sign(0)), so only |Gamma_k| is compared."""
    got, want, y = np.asarray(got), np.asarray(want), np.asarray(y)
    sf = np.asarray(sqrt_f, dtype=np.float64)
    ay = np.abs(y)
    c = (1.0 - eps) / eps
    kappa = np.maximum(1.0, (1.0 + sf / np.where(ay > 0, ay, 1.0)) / (1.0 + lam))
    if lam > c:
        kappa = np.maximum(kappa, c / (lam - c))
    rms = np.sqrt(np.mean(ay.reshape(ay.shape[0], -1) ** 2, axis=1))[:, None, None]
    scale = (ay + rms) * kappa
    diff = np.where(ay > 0, np.abs(got - want), np.abs(np.abs(got) - np.abs(want)))
    scale = np.where(scale > 0, scale, 1.0)
    return float((diff / scale).max())


def lam_rel_operands(got: dict, want: dict, u_new: list, g) -> float:
    """||Lam_gpu - Lam_or|| / || |Lam_or| + |pi u^{n+1}| || over all ordered pairs: the norm
    counterpart of lam_elem_err (Lam is a running sum of differences pi u - v, so its
    rounding scales with u, not with Lam)."""
    num = ref = 0.0
    for (i1, i2, rc) in g.pairs:
        for a, b in ((i1, i2), (i2, i1)):
            pu = u_new[a][g.restrict(a, rc)]
            num += float(np.sum(np.abs(got[(a, b)] - want[(a, b)]) ** 2))
            ref += float(np.sum((np.abs(want[(a, b)]) + np.abs(pu)) ** 2))
    return float(np.sqrt(num / ref)) if ref > 0 else 0.0

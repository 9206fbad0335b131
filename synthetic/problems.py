"""Seeded input recipes (images, probes, scan grids, partitions, Poisson counts).

The paper's own test images and its zone-plate probe are not available, so every
workload is a synthetic stand-in with the paper's shapes (Section 4: a complex
sample built from an amplitude image and a phase image, a small localized probe,
a raster grid scan, Poisson noise controlled by a scaling factor).

Nothing here evaluates the ptychographic forward model; intensities are computed
by the caller's forward operator and only noised here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np
from scipy.ndimage import gaussian_filter


# --------------------------------------------------------------------------
# elementary recipes
# --------------------------------------------------------------------------

def smooth_field(n: int, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """Uniform [0,1) noise, Gaussian-filtered (reflect, truncate 4), min-max scaled to [0,1]."""
    noise = rng.random((n, n))
    s = gaussian_filter(noise, sigma=sigma, mode="reflect", truncate=4.0)
    lo, hi = float(s.min()), float(s.max())
    return (s - lo) / (hi - lo) if hi > lo else np.zeros_like(s)


def make_image(n: int, sigma: float, rng_amp: np.random.Generator,
               rng_phase: np.random.Generator) -> np.ndarray:
    """Complex sample: amplitude 0.5+0.5*s1 and phase (pi/2)*s2 from independent smooth fields."""
    s1 = smooth_field(n, sigma, rng_amp)
    s2 = smooth_field(n, sigma, rng_phase)
    return (0.5 + 0.5 * s1) * np.exp(1j * (np.pi / 2.0) * s2)


def make_probe(p: int, radius: float, quad: float, amplitude: float = 1.0) -> np.ndarray:
    """Disk probe of the given radius about the pixel centre p//2 with quadratic phase quad*r^2.

    An integer centre keeps the probe free of the mirror symmetry about (p-1)/2,
    which would force exact zeros on the Nyquist row and column of F(w) and hence
    ties (y = 0) in the proximal map when the iteration starts from u = 1.
    """
    c = float(p // 2)
    yy, xx = np.mgrid[0:p, 0:p].astype(np.float64)
    r2 = (yy - c) ** 2 + (xx - c) ** 2
    disk = (r2 <= radius * radius).astype(np.float64)
    return amplitude * disk * np.exp(1j * quad * r2)


def raster_positions(n: int, p: int, step: int) -> np.ndarray:
    """Nominal raster positions along one axis, covering [0, n-p].

    If step divides n-p the positions are k*step; otherwise ceil((n-p)/step)+1
    positions are spread evenly (rounded) so the last window touches the edge.
    """
    span = n - p
    if span < 0:
        raise ValueError("probe larger than image")
    if span == 0:
        return np.zeros(1, dtype=np.int64)
    if span % step == 0:
        k = span // step + 1
        return np.arange(k, dtype=np.int64) * step
    k = -(-span // step) + 1
    return np.array([int(round(i * span / (k - 1))) for i in range(k)], dtype=np.int64)


def raster_offsets(n: int, p: int, step: int, jitter: int,
                   rng: Optional[np.random.Generator]) -> tuple[np.ndarray, tuple[int, int]]:
    """Top-left (row, col) of every window on a jittered raster, frames in row-major grid order.

    Jitter is an integer drawn uniformly in [-jitter, jitter] per axis and frame,
    then the offset is clamped to [0, n-p].  Returns (offsets int32 [J,2], (Ky, Kx)).
    """
    pos = raster_positions(n, p, step)
    k = len(pos)
    rows = np.repeat(pos, k).reshape(k, k)
    cols = np.tile(pos, k).reshape(k, k)
    off = np.stack([rows, cols], axis=-1).astype(np.int64)
    if jitter > 0:
        if rng is None:
            raise ValueError("jitter needs a generator")
        off = off + rng.integers(-jitter, jitter + 1, size=off.shape)
    off = np.clip(off, 0, n - p)
    return off.reshape(k * k, 2).astype(np.int32), (k, k)


def _split_sizes(k: int, parts: int) -> list[int]:
    base, rem = divmod(k, parts)
    return [base + (1 if i < rem else 0) for i in range(parts)]


def block_partition(grid: tuple[int, int], dy: int, dx: int) -> np.ndarray:
    """Frame-first partition: the Ky x Kx scan grid cut into dy x dx contiguous blocks.

    Leading blocks take the remainder (25 columns -> 13 + 12).  Subdomain id is
    by*dx + bx.  Returns int32 [Ky*Kx] in the same row-major frame order as
    :func:`raster_offsets`.
    """
    ky, kx = grid
    if not (1 <= dy <= ky and 1 <= dx <= kx):
        raise ValueError("more subdomains than scan rows/columns")
    ry = np.repeat(np.arange(dy), _split_sizes(ky, dy))
    rx = np.repeat(np.arange(dx), _split_sizes(kx, dx))
    sub = ry[:, None] * dx + rx[None, :]
    return sub.reshape(-1).astype(np.int32)


def poisson_counts(intensity: np.ndarray, peak: Optional[float],
                   rng: Optional[np.random.Generator]) -> np.ndarray:
    """Poisson noise with a scaling factor: Poisson(kappa*f)/kappa, kappa = peak/max f.

    ``peak=None`` returns the intensities unchanged (noise-free data).
    """
    f = np.asarray(intensity, dtype=np.float64)
    if peak is None:
        return f.copy()
    fmax = float(f.max())
    if fmax <= 0.0:
        return np.zeros_like(f)
    kappa = peak / fmax
    return rng.poisson(kappa * f).astype(np.float64) / kappa


# --------------------------------------------------------------------------
# workload specifications
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class ProblemSpec:
    """One synthetic ptychography problem (sizes in pixels)."""
    name: str
    n: int                      # image is n x n
    sigma: float                # smoothing of the amplitude/phase fields
    p: int                      # probe is p x p
    radius: float               # true probe disk radius
    quad: float                 # true probe quadratic phase coefficient
    step: int                   # raster step
    jitter: int                 # +- jitter per axis
    dy: int                     # subdomain grid rows (frame blocks)
    dx: int                     # subdomain grid cols
    peak: Optional[float]       # Poisson peak photons; None = noise-free
    iters: int                  # ADMM iterations of the workload
    seed: object = 0            # int or SeedSequence
    blind: bool = False
    init_radius: float = 0.0    # blind: initial flat-phase disk radius
    extra: dict = field(default_factory=dict)


CONFIGS: dict[str, ProblemSpec] = {
    # non-blind, two stripes, FP64-oracle sized
    "c1": ProblemSpec("c1", n=128, sigma=4.0, p=32, radius=12.0, quad=0.02, step=8, jitter=1,
                      dy=1, dx=2, peak=None, iters=50, seed=1),
    # non-blind, 4x4 subdomains, Poisson 1e4 (the throughput workload)
    "c2": ProblemSpec("c2", n=512, sigma=8.0, p=64, radius=24.0, quad=0.02, step=16, jitter=2,
                      dy=4, dx=4, peak=1e4, iters=200, seed=2),
    # amplitude-loss gradient workload (single domain)
    "c3": ProblemSpec("c3", n=1024, sigma=8.0, p=128, radius=48.0, quad=0.01, step=32, jitter=0,
                      dy=1, dx=1, peak=None, iters=1, seed=3),
    # blind, 8x8 subdomains, large
    "c5": ProblemSpec("c5", n=2048, sigma=8.0, p=128, radius=48.0, quad=0.01, step=24, jitter=0,
                      dy=8, dx=8, peak=1e4, iters=300, seed=5, blind=True, init_radius=40.0),
}


def crop_spec(spec: ProblemSpec, n: int, name: Optional[str] = None, **kw) -> ProblemSpec:
    """Same recipe on a smaller image (used for the finite-difference crop and small parity cases)."""
    return replace(spec, name=name or f"{spec.name}_n{n}", n=n, **kw)


def _seed_sequence(seed) -> np.random.SeedSequence:
    if isinstance(seed, np.random.SeedSequence):
        return seed
    return np.random.SeedSequence(int(seed))


def draw_problem(spec: ProblemSpec) -> dict:
    """Draw the sample, probe(s), offsets and partition of a problem.

    Returns a dict with ``u_true`` (complex128 [n,n]), ``w`` (complex128 [p,p], the
    true probe), ``offsets`` (int32 [J,2]), ``grid`` ((Ky,Kx)), ``frame_sub``
    (int32 [J]), ``rng_poisson`` (the generator reserved for noise) and, for blind
    problems, ``w_init_shape`` (the unit-amplitude flat-phase initial disk).
    """
    ss = _seed_sequence(spec.seed)
    s_amp, s_phase, s_jit, s_poi = ss.spawn(4)
    rng_amp = np.random.default_rng(s_amp)
    rng_phase = np.random.default_rng(s_phase)
    rng_jit = np.random.default_rng(s_jit)
    u_true = make_image(spec.n, spec.sigma, rng_amp, rng_phase)
    w = make_probe(spec.p, spec.radius, spec.quad)
    offsets, grid = raster_offsets(spec.n, spec.p, spec.step, spec.jitter, rng_jit)
    frame_sub = block_partition(grid, spec.dy, spec.dx)
    out = dict(spec=spec, u_true=u_true, w=w, offsets=offsets, grid=grid,
               frame_sub=frame_sub, rng_poisson=np.random.default_rng(s_poi))
    if spec.blind:
        out["w_init_shape"] = make_probe(spec.p, spec.init_radius, 0.0)
    return out


def batch_specs(count: int = 64, seed: int = 4) -> list[ProblemSpec]:
    """Uneven batch of independent non-blind problems.

    Per problem: image side uniform over {256,384,...,1024}; probe 64 or 128 (coin
    flip); step = round(p*U(0.25,0.5)); g x g subdomains with g in {2..6}; Poisson
    peak log-uniform in [1e3, 1e5]; 100 iterations.  A grid with more blocks than the
    scan has positions per axis cannot give every subdomain a frame (frame-first
    partition), so g is capped at that count; no other draw is changed.  With
    step >= p/4 a pixel then lies in at most 4 x 4 = 16 subdomains.
    """
    specs = []
    for i, child in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(child.spawn(1)[0])
        n = int(rng.choice(np.arange(256, 1025, 128)))
        p = 64 if rng.random() < 0.5 else 128
        step = int(round(p * rng.uniform(0.25, 0.5)))
        g = int(rng.integers(2, 7))
        peak = float(10.0 ** rng.uniform(3.0, 5.0))
        radius, quad = (24.0, 0.02) if p == 64 else (48.0, 0.01)
        g = min(g, len(raster_positions(n, p, step)))
        specs.append(ProblemSpec(f"c4_{i:02d}", n=n, sigma=8.0, p=p, radius=radius, quad=quad,
                                 step=step, jitter=0, dy=g, dx=g, peak=peak, iters=100,
                                 seed=child))
    return specs


def blind_init_amplitude(sum_intensity_per_frame: float, radius: float) -> float:
    """Flat-disk amplitude whose energy matches the mean frame energy: sqrt(E / (pi R^2))."""
    return math.sqrt(sum_intensity_per_frame / (math.pi * radius * radius))

"""Host-side checks of libodp.so that need no GPU: it loads, exports every symbol
include/odp.h declares, validates its inputs, and its index maps (built in C++)
agree bit for bit with the oracle's independently written geometry.
"""
from __future__ import annotations

import os
import re

import numpy as np
import pytest

import synthetic
import paper_2011_00162_amd as odp
from paper_2011_00162_amd._lib import EXPORTS, OdpError, ODP_EGEOM, ODP_EINVAL, ODP_EUNSUPPORTED
from oracle.geometry import build_geometry, cover_count

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "odp.h")).read()
    declared = set(re.findall(r"\b(odp_[a-z_0-9]+)\s*\(", header))
    assert declared == set(EXPORTS)
    L = odp.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert b"gfx950" in L.odp_version()


def _specs():
    s = [synthetic.CONFIGS[k] for k in ("c1", "c2", "c5")]
    b = synthetic.batch_specs(64)
    s += b[:6] + [b[7], b[14], b[26]]     # 7 and 26: 16 copies of some pixels; 14: 9
    s.append(synthetic.ProblemSpec("paper256", n=256, sigma=4, p=64, radius=24, quad=0.02, step=8,
                                   jitter=0, dy=1, dx=2, peak=None, iters=1, seed=0))
    s.append(synthetic.ProblemSpec("narrow", n=200, sigma=4, p=32, radius=12, quad=0.02, step=6,
                                   jitter=2, dy=3, dx=9, peak=None, iters=1, seed=4))
    return s


@pytest.mark.parametrize("spec", _specs(), ids=lambda s: s.name)
def test_geometry_bit_exact_against_oracle(spec):
    pr = synthetic.draw_problem(spec)
    og = build_geometry(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"])
    plan = odp.Plan(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"], r=1.0, mu=1.0)
    g = plan.geometry()
    np.testing.assert_array_equal(g.rects, og.rects)
    want_pairs = np.array([(a, b, *rc) for (a, b, rc) in og.pairs], dtype=np.int32).reshape(-1, 6)
    np.testing.assert_array_equal(g.pairs, want_pairs)
    np.testing.assert_array_equal(g.cover, cover_count(og))
    assert plan.info.max_cover == int(cover_count(og).max())
    # packed u_sub offsets follow the subdomain order; multiplier storage holds 2 per pair pixel
    sizes = (og.rects[:, 2] - og.rects[:, 0]) * (og.rects[:, 3] - og.rects[:, 1])
    np.testing.assert_array_equal(g.usub_off, np.concatenate([[0], np.cumsum(sizes)[:-1]]))
    areas = [(rc[2] - rc[0]) * (rc[3] - rc[1]) for (_, _, rc) in og.pairs]
    assert plan.info.n_lam == 2 * sum(areas)
    assert plan.info.p_sub == int(sizes.sum())


def test_every_batch_draw_plans_as_drawn():
    """Config 4's 64 draws keep their g x g grids (capped only where the scan has fewer
    positions than blocks); every one makes a plan, whose largest cover, up to 16
    subdomains over a pixel, is the oracle's."""
    covers = []
    for spec in synthetic.batch_specs(64):
        pr = synthetic.draw_problem(spec)
        ky, kx = pr["grid"]
        assert 2 <= spec.dy <= 6 or spec.dy == ky, spec
        og = build_geometry(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"])
        plan = odp.Plan(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"], r=1.0)
        assert plan.info.max_cover == int(cover_count(og).max()) <= 16
        covers.append(plan.info.max_cover)
    assert max(covers) == 16 and sum(c > 8 for c in covers) >= 9


def test_c2_and_c5_pair_counts():
    # 4x4 blocks: 12 horizontal + 12 vertical + 18 diagonal = 42 pairs; 8x8: 210
    for key, want in (("c2", 42), ("c5", 210)):
        spec = synthetic.CONFIGS[key]
        pr = synthetic.draw_problem(spec)
        plan = odp.Plan(spec.n, spec.n, spec.p, pr["offsets"], pr["frame_sub"], r=1.0, mu=1.0)
        assert plan.info.n_pairs == want


def _plan_args(**kw):
    off, grid = synthetic.raster_offsets(64, 32, 8, 0, None)
    sub = synthetic.block_partition(grid, 1, 2)
    a = dict(H=64, W=64, p=32, offsets=off, frame_sub=sub, eps=0.5, eta=0.1, r=1.0)
    a.update(kw)
    return a


@pytest.mark.parametrize("kw,code", [
    (dict(eps=1.0), ODP_EINVAL),
    (dict(eps=0.0), ODP_EINVAL),
    (dict(eta=0.0), ODP_EINVAL),
    (dict(r=0.0), ODP_EINVAL),
    (dict(p=48), ODP_EUNSUPPORTED),
    (dict(H=16), ODP_EINVAL),
    (dict(blind=True, mu=0.0), ODP_EINVAL),                        # blind needs mu > 0
    (dict(gamma=-1.0), ODP_EINVAL),
    (dict(transform=odp.ODP_DFT_SPLIT_BF16), ODP_EUNSUPPORTED),     # the MFMA transform is for p = 64
])
def test_plan_rejects_bad_parameters(kw, code):
    with pytest.raises(OdpError) as e:
        odp.Plan(**_plan_args(**kw))
    assert e.value.code == code


def test_plan_rejects_bad_geometry():
    a = _plan_args()
    off = a["offsets"].copy()
    off[2, 1] = 40          # 40 + 32 > 64
    with pytest.raises(OdpError) as e:
        odp.Plan(**{**a, "offsets": off})
    assert e.value.code == ODP_EGEOM
    sub = a["frame_sub"].copy()
    with pytest.raises(OdpError) as e:
        odp.Plan(**{**a, "frame_sub": np.where(sub == 1, 2, sub), "D": 3})   # subdomain 1 empty
    assert e.value.code == ODP_EGEOM
    with pytest.raises(OdpError) as e:
        odp.Plan(**{**a, "frame_sub": sub + 5, "D": 2})
    assert e.value.code == ODP_EGEOM


def test_degenerate_scans_are_refused():
    """No frames, a window with a negative offset, an empty batch: refused on the host."""
    a = _plan_args()
    with pytest.raises(OdpError) as e:
        odp.Plan(**{**a, "offsets": np.zeros((0, 2), np.int32), "frame_sub": np.zeros(0, np.int32)})
    assert e.value.code == ODP_EINVAL
    off = a["offsets"].copy()
    off[0, 1] = -1
    with pytest.raises(OdpError) as e:
        odp.Plan(**{**a, "offsets": off})
    assert e.value.code == ODP_EGEOM
    with pytest.raises(OdpError) as e:
        odp.Plan.batch([])
    assert e.value.code == ODP_EINVAL


def test_one_subdomain_needs_no_overlap_penalty():
    a = _plan_args(r=0.0, frame_sub=np.zeros(len(_plan_args()["offsets"]), np.int32))
    plan = odp.Plan(**a)
    assert plan.info.D == 1 and plan.info.n_pairs == 0 and plan.info.n_lam == 0


def _batch_problems(n=5):
    out = []
    for s in synthetic.batch_specs(64)[:n]:
        pr = synthetic.draw_problem(s)
        out.append((s, pr))
    return out


def test_batch_plan_packs_independent_problems():
    items = [(s, pr) for (s, pr) in _batch_problems(8) if s.p == 64]
    probs = [dict(H=s.n, W=s.n, p=s.p, offsets=pr["offsets"], frame_sub=pr["frame_sub"], r=1.0 + i)
             for i, (s, pr) in enumerate(items)]
    batch = odp.Plan.batch(probs)
    g = batch.geometry()
    assert batch.n_problems() == len(items)
    pair_rows = []
    for i, (s, pr) in enumerate(items):
        e = batch.entry(i)
        single = odp.Plan(s.n, s.n, s.p, pr["offsets"], pr["frame_sub"], r=1.0)
        sg = single.geometry()
        # rectangles shifted by the problem's column origin
        want = sg.rects + np.array([0, e.col0, 0, e.col0], dtype=np.int32)
        np.testing.assert_array_equal(g.rects[e.D0:e.D0 + e.D], want)
        for q in sg.pairs:
            pair_rows.append((q[0] + e.D0, q[1] + e.D0, q[2], q[3] + e.col0, q[4], q[5] + e.col0))
        assert e.r == 1.0 + i and e.J == len(pr["offsets"])
    # no pair crosses problems
    np.testing.assert_array_equal(g.pairs, np.array(sorted(pair_rows), dtype=np.int32).reshape(-1, 6))


def test_batch_cells_are_the_problems_own():
    """Each problem of a batch is cut into pixel-update cells at its own subdomain edges
    only: the batch's cells and tiles are those of its problems planned alone, at every
    tiling (cutting at the other problems' edges too multiplied them about 17-fold)."""
    items = [(s, pr) for (s, pr) in _batch_problems(12) if s.p == 64]
    probs = [dict(H=s.n, W=s.n, p=s.p, offsets=pr["offsets"], frame_sub=pr["frame_sub"], r=1.0) for s, pr in items]
    batch = odp.Plan.batch(probs)
    singles = [odp.Plan(s.n, s.n, s.p, pr["offsets"], pr["frame_sub"], r=1.0) for s, pr in items]
    assert batch.info.n_cells == sum(q.info.n_cells for q in singles)
    L = odp.lib()
    for tiling in (0, 1, 2):
        for q in [batch] + singles:
            assert L.odp_plan_set_tuning(q._h, odp.ODP_FFT_F32, 0, tiling, None) == 0
        assert batch.info.n_tiles == sum(q.info.n_tiles for q in singles), tiling


def test_batch_rejects_mixed_probe_sizes():
    items = _batch_problems(12)
    ps = {s.p for s, _ in items}
    assert ps == {64, 128}
    probs = [dict(H=s.n, W=s.n, p=s.p, offsets=pr["offsets"], frame_sub=pr["frame_sub"], r=1.0) for s, pr in items]
    with pytest.raises(OdpError):
        odp.Plan.batch(probs)


def test_sweep_event_arguments_are_checked():
    import ctypes as C
    plan = odp.Plan(**_plan_args())
    L = odp.lib()
    one = (C.c_void_p * 1)(C.c_void_p(0x1000))
    nul = (C.c_void_p * 1)(None)
    assert L.odp_plan_set_sweep_events(plan._h, None, None, 0, 1) == 0          # cancel
    assert L.odp_plan_set_sweep_events(plan._h, None, None, -1, 1) == ODP_EINVAL
    assert L.odp_plan_set_sweep_events(plan._h, one, one, 1, 0) == ODP_EINVAL   # stride < 1
    assert L.odp_plan_set_sweep_events(plan._h, None, one, 1, 1) == ODP_EINVAL  # null array
    assert L.odp_plan_set_sweep_events(plan._h, nul, one, 1, 1) == ODP_EINVAL   # null event
    assert L.odp_plan_set_sweep_events(plan._h, None, None, 0, 1) == 0


def test_tuning_values_are_checked():
    plan = odp.Plan(**_plan_args())
    L = odp.lib()
    assert L.odp_plan_set_tuning(plan._h, odp.ODP_FFT_F32, 3, 0, None) == ODP_EINVAL
    assert L.odp_plan_set_tuning(plan._h, odp.ODP_FFT_F32, -1, 0, None) == ODP_EINVAL
    assert L.odp_plan_set_tuning(plan._h, odp.ODP_FFT_F32, 0, 3, None) == ODP_EINVAL
    for xcd in (0, 1, 2):
        for tiling, shape in ((0, (16, 32)), (1, (8, 64)), (2, (32, 16))):
            assert L.odp_plan_set_tuning(plan._h, odp.ODP_FFT_F32, xcd, tiling, None) == 0   # unbound: host only
            t = plan.tuning()
            assert (t.xcd_slice, t.tiling, (t.tile_rows, t.tile_cols)) == (xcd, tiling, shape)


def test_pixel_pairs_follow_the_window_columns():
    """The paired pull (one 16-byte load for a thread's two row neighbours) is on exactly
    when every window of a tile starts at a column of the tile's parity: even raster
    offsets give even cell edges; one window moved to an odd column turns it off."""
    L = odp.lib()
    plan = odp.Plan(**_plan_args())                       # offsets 0, 8, ..., 32: all even
    for tiling in (0, 1, 2):
        assert L.odp_plan_set_tuning(plan._h, odp.ODP_FFT_F32, 0, tiling, None) == 0
        assert plan.tuning().pixel_pairs == 1
    plan.set_pixel_pairs(0)
    assert plan.tuning().pixel_pairs == 0
    plan.set_pixel_pairs(1)
    assert plan.tuning().pixel_pairs == 1
    assert L.odp_plan_set_pixel_pairs(plan._h, 2) == ODP_EINVAL
    assert L.odp_plan_set_pixel_pairs(plan._h, -1) == ODP_EINVAL
    assert L.odp_plan_set_pixel_pairs(None, 1) == ODP_EINVAL
    a = _plan_args()
    off = a["offsets"].copy()
    off[5, 1] += 1                                        # one window of the first subdomain at an odd column
    a["offsets"] = off
    odd = odp.Plan(**a)
    for tiling in (0, 1, 2):
        assert L.odp_plan_set_tuning(odd._h, odp.ODP_FFT_F32, 0, tiling, None) == 0
        assert odd.tuning().pixel_pairs == 0


def test_initial_probe_arguments_are_checked():
    import ctypes as C
    plan = odp.Plan(**_plan_args())
    L = odp.lib()
    assert L.odp_blind_initial_probe(None, C.c_void_p(0x1000), None) == ODP_EINVAL   # null plan
    assert L.odp_blind_initial_probe(plan._h, None, None) == ODP_EINVAL              # null output
    assert L.odp_blind_initial_probe(plan._h, C.c_void_p(0x1000), None) == ODP_EINVAL   # not bound


def test_stopping_arguments_are_checked():
    plan = odp.Plan(**_plan_args())
    L = odp.lib()
    assert L.odp_plan_set_stopping(None, odp.ODP_STOP_RF, 1e-5, 1000, 1) == ODP_EINVAL
    assert L.odp_plan_set_stopping(plan._h, 3, 1e-5, 0, 1) == ODP_EINVAL           # unknown measure
    assert L.odp_plan_set_stopping(plan._h, -1, 1e-5, 0, 1) == ODP_EINVAL
    assert L.odp_plan_set_stopping(plan._h, odp.ODP_STOP_RE, -1e-3, 0, 1) == ODP_EINVAL
    assert L.odp_plan_set_stopping(plan._h, odp.ODP_STOP_RE, float("nan"), 0, 1) == ODP_EINVAL
    assert L.odp_plan_set_stopping(plan._h, odp.ODP_STOP_RE, 1e-3, -1, 1) == ODP_EINVAL
    # the paper's two rules and a bare cap (host-side settings: no device needed)
    assert L.odp_plan_set_stopping(plan._h, odp.ODP_STOP_RF, 1e-5, 1000, 1) == 0
    assert L.odp_plan_set_stopping(plan._h, odp.ODP_STOP_RE, 1e-3, 200, 1) == 0
    assert L.odp_plan_set_stopping(plan._h, odp.ODP_STOP_NONE, float("nan"), 7, 1) == 0
    assert L.odp_plan_set_stopping(plan._h, odp.ODP_STOP_NONE, 0.0, 0, 1) == 0
    assert L.odp_plan_set_stopping(plan._h, odp.ODP_STOP_RE, 1e-3, 200, 0) == ODP_EINVAL   # check interval < 1
    assert L.odp_plan_set_stopping(plan._h, odp.ODP_STOP_RE, 1e-3, 200, 10) == 0


def test_balancing_arguments_are_checked():
    plan = odp.Plan(**_plan_args())
    L = odp.lib()
    assert L.odp_plan_set_balancing(None, 10.0, 2.0, 10, 0, 1) == ODP_EINVAL
    assert L.odp_plan_set_balancing(plan._h, 10.0, 2.0, -1, 0, 1) == ODP_EINVAL      # negative period
    assert L.odp_plan_set_balancing(plan._h, 10.0, 2.0, 10, -1, 1) == ODP_EINVAL     # negative limit
    assert L.odp_plan_set_balancing(plan._h, 0.5, 2.0, 10, 0, 1) == ODP_EINVAL       # mu < 1
    assert L.odp_plan_set_balancing(plan._h, 10.0, 1.0, 10, 0, 1) == ODP_EINVAL      # tau <= 1
    assert L.odp_plan_set_balancing(plan._h, 10.0, float("inf"), 10, 0, 1) == ODP_EINVAL
    assert L.odp_plan_set_balancing(plan._h, float("nan"), 2.0, 10, 0, 1) == ODP_EINVAL
    assert L.odp_plan_set_balancing(plan._h, 10.0, 2.0, 10, 500, 1) == 0
    assert L.odp_plan_set_balancing(plan._h, float("inf"), 2.0, 1, 0, 1) == 0      # never triggers
    assert L.odp_plan_set_balancing(plan._h, 0.0, 0.0, 0, 0, 1) == 0                  # off: values unchecked
    assert L.odp_plan_set_balancing(plan._h, 10.0, 2.0, 10, 0, 0) == ODP_EINVAL       # nothing selected
    assert L.odp_plan_set_balancing(plan._h, 10.0, 2.0, 10, 0, 4) == ODP_EINVAL
    assert L.odp_plan_set_balancing(plan._h, 10.0, 2.0, 10, 0, 3) == 0                # r and eta
    assert L.odp_plan_get_eta(plan._h) == plan.params["eta"] and L.odp_plan_get_eta(None) == 0.0


def test_size_helpers_match_plan_info():
    plan = odp.Plan(**_plan_args())
    L = odp.lib()
    assert L.odp_plan_workspace_bytes(plan._h) == plan.info.workspace_bytes > 0
    assert L.odp_state_bytes(plan._h) == plan.info.state_bytes > 0
    assert L.odp_plan_workspace_bytes(None) == 0 and L.odp_state_bytes(None) == 0


def test_batches_hold_known_probe_problems_only():
    items = [(s, pr) for (s, pr) in _batch_problems(8) if s.p == 64][:2]
    probs = [dict(H=s.n, W=s.n, p=s.p, offsets=pr["offsets"], frame_sub=pr["frame_sub"], r=1.0) for s, pr in items]
    probs[1].update(blind=True, mu=1.0)
    with pytest.raises(OdpError) as e:
        odp.Plan.batch(probs)
    assert e.value.code == ODP_EUNSUPPORTED


def test_eta_balancing_is_refused_for_blind_plans():
    plan = odp.Plan(**_plan_args(blind=True, mu=1.0))
    L = odp.lib()
    assert L.odp_plan_set_balancing(plan._h, 10.0, 2.0, 4, 0, odp.ODP_BALANCE_ETA) == ODP_EUNSUPPORTED
    assert L.odp_plan_set_balancing(plan._h, 10.0, 2.0, 4, 0, odp.ODP_BALANCE_R) == 0


def test_benchmark_reads_measured_traffic_only_for_the_current_kernels(tmp_path):
    """A PMC summary's traffic is used only while its kernel-source hash matches; the
    known-probe and blind lines are read by their own keys."""
    import bench
    good = tmp_path / "good.md"
    good.write_text("traffic_bytes_per_launch: 1.5e+09\ntraffic_bytes_per_launch_blind: 2.5e+09\n"
                    f"kernel_source_sha256_16: {bench.kernel_hash()}\n")
    assert bench.measured_traffic(str(good)) == 1.5e9
    assert bench.measured_traffic(str(good), "traffic_bytes_per_launch_blind") == 2.5e9
    stale = tmp_path / "stale.md"
    stale.write_text("traffic_bytes_per_launch: 1.5e+09\nkernel_source_sha256_16: 0000000000000000\n")
    assert bench.measured_traffic(str(stale)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md")) is None

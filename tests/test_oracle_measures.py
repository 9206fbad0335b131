"""Pins of the oracle's Sec. 4 measures and merge on hand-computed cases.

Each expected value below is worked out by hand from the definitions in Sec. 4 (the
R-factor RF, the relative error RE, the SNR of a recovery u_r against a ground truth u_g
with ||u_r||^2 in its denominator, and the merge that keeps non-overlapping pixels and
averages overlaps), on arrays small enough to check on paper.  The cases are chosen so
that the plausible slips (an L2 norm for an L1 norm, f for sqrt f, the old iterate's norm
in RE, keeping one copy instead of averaging, the truth's norm in the SNR) give another
number.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle.geometry import Geometry
from oracle.od2p import merge, r_factor, relative_change, snr_db


def test_r_factor_hand_computed():
    # two frames of 1 x 2: |X| = [[5, 0], [1, 2]], sqrt f = [[4, 1], [2, 2]]
    X = np.array([[[3 + 4j, 0]], [[1j, -2]]])
    sf = np.array([[[4.0, 1.0]], [[2.0, 2.0]]])
    # sum | |X| - sqrt f | = 1 + 1 + 1 + 0 = 3 and sum sqrt f = 9
    assert r_factor(X, sf) == pytest.approx(1.0 / 3.0, rel=1e-15)
    # an L2 reading would give sqrt(3) / sqrt(25); f in place of sqrt f another value
    assert not math.isclose(r_factor(X, sf), math.sqrt(3.0) / 5.0, rel_tol=1e-3)
    assert not math.isclose(r_factor(X, sf), 3.0 / 25.0, rel_tol=1e-3)   # f = sqrt(f)^2 in the denominator


def test_r_factor_zero_only_at_the_data():
    X = np.array([[[2.0, -1j]]])
    assert r_factor(X, np.array([[[2.0, 1.0]]])) == 0.0
    assert r_factor(X, np.array([[[1.0, 1.0]]])) == pytest.approx(0.5, rel=1e-15)   # |2 - 1| / 2


def test_relative_change_hand_computed():
    # subdomain 0: ||u^n - u^{n-1}|| = |1j| = 1, ||u^n|| = sqrt(1 + 2) -> 1/sqrt(3)
    # subdomain 1: unchanged -> 0; RE is the max over subdomains
    old = [np.array([[1.0 + 0j, 1.0]]), np.array([[2.0 + 0j]])]
    new = [np.array([[1.0 + 0j, 1.0 + 1j]]), np.array([[2.0 + 0j]])]
    assert relative_change(old, new) == pytest.approx(1.0 / math.sqrt(3.0), rel=1e-15)
    # dividing by ||u^{n-1}|| = sqrt 2 would give 1/sqrt(2)
    assert not math.isclose(relative_change(old, new), 1.0 / math.sqrt(2.0), rel_tol=1e-3)
    # the max picks the second subdomain: ||(3, 4i) - 0|| / ||(3, 4i)|| = 1 (the old norm is 0)
    old2 = [old[0], np.zeros((1, 2), complex)]
    new2 = [new[0], np.array([[3.0 + 0j, 4j]])]
    assert relative_change(old2, new2) == pytest.approx(1.0, rel=1e-15)


def _strip_geometry():
    # image 1 x 5; subdomain 0 covers columns [0, 3), subdomain 1 columns [1, 4); column 4 is
    # in no subdomain
    rects = np.array([[0, 0, 1, 3], [0, 1, 1, 4]], dtype=np.int64)
    return Geometry(h=1, w=5, p=1, offsets=np.zeros((2, 2), np.int64), frame_sub=np.array([0, 1]),
                    rects=rects, pairs=[(0, 1, (0, 1, 1, 3))], frames_of=[np.array([0]), np.array([1])])


def test_merge_keeps_single_copies_and_averages_overlaps():
    g = _strip_geometry()
    u0 = np.array([[1.0 + 0j, 2.0, 3.0]])
    u1 = np.array([[10j, 20.0, 30.0]])
    got = merge(g, [u0, u1])
    # column 0 only in u0; columns 1, 2 averaged: (2 + 10i)/2, (3 + 20)/2; column 3 only in
    # u1; column 4 uncovered -> 1
    want = np.array([[1.0, 1.0 + 5j, 11.5, 30.0, 1.0]])
    np.testing.assert_array_equal(got, want)
    assert merge(g, [u0, u1], fill=0.0)[0, 4] == 0.0


def test_snr_hand_computed():
    # u_r = (1, i), u_g = (1, 0): the best phase is 0; ||u_r - u_g||^2 = 1, ||u_r||^2 = 2
    ur = np.array([1.0 + 0j, 1j])
    ug = np.array([1.0 + 0j, 0.0])
    assert snr_db(ur, ug) == pytest.approx(10.0 * math.log10(2.0), rel=1e-13)
    # a global phase of the recovery changes nothing
    assert snr_db(ur * np.exp(0.7j), ug) == pytest.approx(10.0 * math.log10(2.0), rel=1e-12)
    # u_r = 2 u_g: ||u_r - u_g||^2 = ||u_g||^2 and ||u_r||^2 = 4 ||u_g||^2 -> 10 log10 4; with
    # the truth's norm in the denominator it would be 0 dB
    ug2 = np.array([1.0 + 1j, -2.0, 0.5j])
    assert snr_db(2.0 * ug2, ug2) == pytest.approx(10.0 * math.log10(4.0), rel=1e-13)
    assert snr_db(0.5 * ug2, ug2) == pytest.approx(0.0, abs=1e-13)

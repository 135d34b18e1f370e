"""Best-candidate lattices (section "Generating a Lattice", second method): the oracle pinned
against library k-nearest-neighbour and pair searches, and the native builder bit-exact
against the oracle."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import workloads as W
from oracle import candidate as OC
from paper_2207_09334_amd import cronos as CR

SIZE = (0.1, 0.03, 0.02)


def test_one_candidate_per_point_gives_the_draws():
    """With a single candidate there is no choice: point p is the draw (seed, 8, p, 0, axis)."""
    pts = OC.best_candidate_points(SIZE, 40, n_candidates=1, k_nn=3, seed=7)
    p = np.arange(40)[:, None]
    a = np.arange(3)[None, :]
    np.testing.assert_array_equal(pts, np.asarray(SIZE)[None, :] * W.uniform01(7, W.S_CANDIDATE, p, 0, a))


@pytest.mark.parametrize("k_nn", [1, 4])
def test_each_point_is_the_best_candidate_by_kdtree(k_nn):
    """Every placed point is one of its step's candidates and has the largest sum of its
    k nearest-neighbour distances among them (scipy's k-d tree as the independent search)."""
    n, C, seed = 120, 100, 3
    pts = OC.best_candidate_points(SIZE, n, C, k_nn, seed)
    c = np.arange(C)[:, None]
    a = np.arange(3)[None, :]
    for p in range(1, n):
        cand = np.asarray(SIZE)[None, :] * W.uniform01(seed, W.S_CANDIDATE, p, c, a)
        k = min(k_nn, p)
        d, _ = cKDTree(pts[:p]).query(cand, k=k)
        score = d.reshape(C, k).sum(axis=1)
        hit = np.nonzero((cand == pts[p]).all(axis=1))[0]
        assert len(hit) >= 1
        assert score[hit[0]] >= score.max() * (1 - 1e-12)


def test_quasi_uniform_spacing():
    """Best-candidate points (k = 1: Mitchell's nearest-distance criterion, the one that
    targets a minimum spacing) keep a minimum distance several times that of uniform points."""
    n = 400
    pts = OC.best_candidate_points(SIZE, n, 100, 1, seed=1)
    rnd = np.asarray(SIZE)[None, :] * W.uniform01(1, W.S_CANDIDATE, np.arange(n)[:, None], 0, np.arange(3)[None, :])
    dmin = lambda x: cKDTree(x).query(x, k=2)[0][:, 1].min()
    spacing = (np.prod(SIZE) / n) ** (1 / 3)
    assert dmin(pts) > 0.3 * spacing
    assert dmin(pts) > 5 * dmin(rnd)


def test_cutoff_springs_match_kdtree_pairs():
    pts = OC.best_candidate_points(SIZE, 300, 100, 4, seed=2)
    r = 1.6 * (np.prod(SIZE) / 300) ** (1 / 3)
    ends = OC.cutoff_springs(pts, r)
    ref = np.array(sorted(cKDTree(pts).query_pairs(r)))
    # the pair search is the library's; only pairs at the cutoff within rounding may differ
    d = np.linalg.norm(pts[ends[:, 0]] - pts[ends[:, 1]], axis=1)
    assert set(map(tuple, ends.tolist())) ^ set(map(tuple, ref.tolist())) <= {
        tuple(e) for e, dd in zip(ends.tolist(), d) if abs(dd - r) < 1e-12 * r}
    assert (ends[:, 0] < ends[:, 1]).all()


@pytest.mark.parametrize("n,k_nn,seed", [(50, 1, 0), (400, 4, 1), (700, 8, 2)])
def test_native_points_and_springs_bit_exact(n, k_nn, seed):
    a = OC.best_candidate_points(SIZE, n, 100, k_nn, seed)
    b = CR.cronos_candidate_points(SIZE, n, 100, k_nn, seed)
    np.testing.assert_array_equal(a, b)
    r = 1.6 * (np.prod(SIZE) / n) ** (1 / 3)
    np.testing.assert_array_equal(OC.cutoff_springs(a, r), CR.cronos_cutoff_springs(b, r))


def test_native_candidate_rejects_bad_arguments():
    with pytest.raises(CR.CronosError):
        CR.cronos_candidate_points((0.1, 0.0, 0.1), 10)
    with pytest.raises(CR.CronosError):
        CR.cronos_candidate_points(SIZE, 10, k_nn=0)
    with pytest.raises(CR.CronosError):
        CR.cronos_cutoff_springs(np.zeros((3, 3)), -1.0)


def test_native_point_params_bit_exact():
    """The library's spring parameters of a point lattice (rest = initial length, k scaled
    inversely to it, uniform mass, the x < pin_x end fixed) equal the oracle system's bit for
    bit; every rest length is the pair's distance."""
    pw = W.candidate_bar(600, size=SIZE, seed=3)
    pts = OC.best_candidate_points(pw.size, pw.n_points, pw.n_candidates, pw.k_nn, pw.seed)
    ends = OC.cutoff_springs(pts, pw.cutoff)
    ref = OC.system(pw, pts, ends)
    k, rest, mass, pinned = CR.cronos_point_params(pts, ends, pw.k_ref, pw.length_ref, pw.mass, pin_axis=0,
                                                   pin_below=pw.pin_x)
    np.testing.assert_array_equal(rest, ref.rest)
    np.testing.assert_array_equal(k, ref.k)
    np.testing.assert_array_equal(mass, ref.mass)
    np.testing.assert_array_equal(pinned.astype(bool), ref.pinned)
    assert 0 < pinned.sum() < len(pts)
    np.testing.assert_allclose(rest, np.linalg.norm(pts[ends[:, 1]] - pts[ends[:, 0]], axis=1), rtol=1e-15)
    np.testing.assert_allclose(k * rest, pw.k_ref * pw.length_ref, rtol=1e-15)
    _, _, _, none = CR.cronos_point_params(pts, ends, 1.0, 1.0, 1.0)
    assert not none.any()
    with pytest.raises(CR.CronosError):
        CR.cronos_point_params(pts, np.array([[0, 0]]), 1.0, 1.0, 1.0)
    with pytest.raises(CR.CronosError):
        CR.cronos_point_params(pts, np.array([[0, len(pts)]]), 1.0, 1.0, 1.0)
    with pytest.raises(CR.CronosError):
        CR.cronos_point_params(pts, ends, 1.0, 1.0, 1.0, pin_axis=3)

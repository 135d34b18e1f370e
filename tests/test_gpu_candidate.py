"""GPU parity on a best-candidate lattice (section "Generating a Lattice", second method):
irregular degrees, float-coordinate Morton keys, distance-cutoff springs (run on an MI355X).
The oracle builds its own points and springs (bit-exact with the native builder) and steps
them in FP64; the same bars as the voxel lattices."""
import numpy as np
import pytest

import workloads as W
from oracle import candidate as OC
from oracle import layout as LY
from oracle import physics as P
from paper_2207_09334_amd import cronos as CR
from paper_2207_09334_amd import problem as PR
from tests.gpu_common import force_error, position_error, say

pytestmark = pytest.mark.gpu

F_TOL = 1e-5
X_TOL = 1e-4


def _pair(n=2000):
    pw = W.candidate_bar(n, size=(0.1, 0.02, 0.02), seed=9)
    pts = OC.best_candidate_points(pw.size, pw.n_points, pw.n_candidates, pw.k_nn, pw.seed)
    ends = OC.cutoff_springs(pts, pw.cutoff)
    sys_ = OC.system(pw, pts, ends)
    sim, npts, nends, _, _ = PR.create_points(pw, flags=CR.CHECK_LAYOUT)
    assert np.array_equal(npts, pts) and np.array_equal(nends, ends)
    return pw, pts, ends, sys_, sim


def test_candidate_bar_forces_and_positions():
    pw, pts, ends, sys_, sim = _pair()
    degree = np.bincount(ends.ravel(), minlength=len(pts))
    say(f"case: best-candidate bar, {len(pts)} points, {len(ends)} springs, degree {degree.min()}-{degree.max()}")
    x, v = pts.copy(), np.zeros_like(pts)
    worst = 0.0
    for n in range(0, 1000, 100):
        x, v = P.run(sys_, x, v, n, 100)
        CR.cronos_step(sim, 100)
        xg, _, _ = CR.cronos_read_state(sim)
        worst = max(worst, position_error(xg, x))
        if n == 200:
            e, _ = force_error(CR.cronos_eval_forces(sim), sys_, xg, 300 * pw.dt)
            say(f"  force err at step 300 {e:.2e}")
            assert e <= F_TOL
    say(f"  position err over 1000 steps {worst:.3e}")
    assert worst <= X_TOL


def test_candidate_layout_matches_oracle():
    pw, pts, ends, sys_, sim = _pair(1500)
    got = CR.cronos_get_layout(sim)
    ora = LY.reorder(ends, np.array([0, len(pts)]), x=pts)
    for f in ("perm", "row_ptr", "col", "sid", "spring_perm"):
        assert np.array_equal(got[f], getattr(ora, f))

"""Tangent stiffness and natural frequencies, FP64 (test infrastructure).

Section "Natural Frequency Analysis" predicts a structure's natural frequencies from the
generalised eigenproblem K v = w^2 M v with a mass matrix M and a stiffness matrix K.  Here
K is the tangent stiffness of the Hookean springs of eq. (2): for a spring with unit
direction n, length l and rest length l0 the 3x3 block is
    K_s = k [ n n^T + (1 - l0 / l) (I - n n^T) ],
entering the (i,i), (j,j) blocks with + and the (i,j), (j,i) blocks with -; so that
df = -K dx.  M is the diagonal lumped mass matrix.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import physics


def spring_blocks(x: np.ndarray, ends: np.ndarray, k: np.ndarray, l0: np.ndarray) -> np.ndarray:
    """(S, 3, 3) tangent stiffness block of each spring."""
    d, length = physics.spring_vectors(x, ends)
    n = d / length[:, None]
    nn = n[:, :, None] * n[:, None, :]
    eye = np.eye(3)[None]
    return k[:, None, None] * (nn + (1.0 - l0 / length)[:, None, None] * (eye - nn))


def stiffness(x: np.ndarray, ends: np.ndarray, k: np.ndarray, l0: np.ndarray) -> sp.csr_matrix:
    """Sparse 3N x 3N tangent stiffness K with df = -K dx."""
    N = len(x)
    B = spring_blocks(x, ends, k, l0)
    i, j = ends[:, 0], ends[:, 1]
    r, c, v = [], [], []
    for a in range(3):
        for b in range(3):
            blk = B[:, a, b]
            for (ri, ci, sgn) in ((i, i, 1.0), (j, j, 1.0), (i, j, -1.0), (j, i, -1.0)):
                r.append(3 * ri + a)
                c.append(3 * ci + b)
                v.append(sgn * blk)
    return sp.csr_matrix((np.concatenate(v), (np.concatenate(r), np.concatenate(c))), shape=(3 * N, 3 * N))


def contact_stiffness(x: np.ndarray, ground_z: float, ground_k: float) -> sp.csr_matrix:
    """Tangent stiffness of the penalty contact plane (Appendix A's contact planes, normal force
    k_g max(0, z_g - z) on +z): k_g on the z diagonal of every mass below the plane."""
    N = len(x)
    d = np.zeros(3 * N)
    d[2::3] = np.where(x[:, 2] < ground_z, ground_k, 0.0)
    return sp.diags(d).tocsr()


def free_dofs(pinned: np.ndarray) -> np.ndarray:
    return np.nonzero(np.repeat(~np.asarray(pinned, bool), 3))[0]


def static_displacement(x, ends, k, l0, pinned, f) -> np.ndarray:
    """Solve K u = f on the free degrees of freedom (pinned masses fixed)."""
    K = stiffness(x, ends, k, l0)
    dof = free_dofs(pinned)
    u = np.zeros(3 * len(x))
    u[dof] = spla.spsolve(K[dof][:, dof].tocsc(), np.asarray(f).ravel()[dof])
    return u.reshape(-1, 3)


def natural_frequencies(x, ends, k, l0, mass, pinned, count: int = 2, ground=None):
    """Smallest ``count`` angular frequencies w (rad/s) and mode shapes of K v = w^2 M v,
    found by shift-invert Lanczos around zero (a sparse factorisation of K).  ground =
    (z_g, k_g) adds the contact plane's stiffness to K."""
    K = stiffness(x, ends, k, l0)
    if ground is not None:
        K = (K + contact_stiffness(x, ground[0], ground[1])).tocsr()
    dof = free_dofs(pinned)
    Kf = K[dof][:, dof].tocsc()
    Mf = sp.diags(np.repeat(mass, 3)[dof]).tocsc()
    # a fixed start vector: ARPACK's own draws from a generator that earlier calls advance,
    # so within a degenerate eigenspace the returned vectors would depend on call history
    v0 = np.random.default_rng(12345).uniform(-1.0, 1.0, len(dof))
    w2, vec = spla.eigsh(Kf, k=count, M=Mf, sigma=0.0, which="LM", v0=v0)
    order = np.argsort(w2)
    modes = np.zeros((count, 3 * len(x)))
    modes[:, dof] = vec[:, order].T
    return np.sqrt(w2[order]), modes.reshape(count, -1, 3)

"""Seeded synthetic inputs shared by the tests, the bench and the smoke check.

This module holds no arithmetic of the CTMRG method: it only produces the
model's spin vectors (the vertices of the regular polyhedra, Sec. I of the
paper) and seeded random states/matrices for kernel tests.  Both the CPU
oracle and the GPU library receive these as plain arrays.

Vertex order convention: vertex 0 is the boundary spin of the fixed boundary
condition (the paper's "s = 1", Sec. II).  Sign patterns are enumerated with +
before -, so vertex 0 of the cube and the dodecahedron is (1,1,1)/sqrt(3).
"""
from __future__ import annotations

import itertools

import numpy as np

GOLDEN = (1.0 + 5.0 ** 0.5) / 2.0


def _signs(k):
    return list(itertools.product((1.0, -1.0), repeat=k))


def _normalize(rows):
    v = np.asarray(rows, dtype=np.float64)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def ising():
    """q=2 spins +1/-1 as one-dimensional unit vectors."""
    return np.array([[1.0], [-1.0]])


def square():
    """q=4 unit vectors at 0, 90, 180, 270 degrees."""
    return np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0]])


def tetrahedron():
    """q=4 vertices of the regular tetrahedron inscribed in the cube."""
    return _normalize([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]])


def octahedron():
    """q=6 vertices +-e_x, +-e_y, +-e_z."""
    return np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0], [0, 0, 1.0], [0, 0, -1.0]])


def cube():
    """q=8 vertices (+-1,+-1,+-1)/sqrt(3)."""
    return _normalize(_signs(3))


def icosahedron():
    """q=12 vertices (0,+-1,+-phi), (+-1,+-phi,0), (+-phi,0,+-1), normalized."""
    rows = []
    for a, b in _signs(2):
        rows.append([0.0, a, b * GOLDEN])
    for a, b in _signs(2):
        rows.append([a, b * GOLDEN, 0.0])
    for a, b in _signs(2):
        rows.append([a * GOLDEN, 0.0, b])
    return _normalize(rows)


def dodecahedron():
    """q=20 vertices (+-1,+-1,+-1), (0,+-1/phi,+-phi), (+-1/phi,+-phi,0), (+-phi,0,+-1/phi), over sqrt(3)."""
    rows = [list(s) for s in _signs(3)]
    ip = 1.0 / GOLDEN
    for a, b in _signs(2):
        rows.append([0.0, a * ip, b * GOLDEN])
    for a, b in _signs(2):
        rows.append([a * ip, b * GOLDEN, 0.0])
    for a, b in _signs(2):
        rows.append([a * GOLDEN, 0.0, b * ip])
    return np.asarray(rows, dtype=np.float64) / np.sqrt(3.0)


MODELS = {
    "ising": ising,
    "square": square,
    "tetrahedron": tetrahedron,
    "octahedron": octahedron,
    "cube": cube,
    "icosahedron": icosahedron,
    "dodecahedron": dodecahedron,
}


def vertices(name: str) -> np.ndarray:
    return MODELS[name]()


def random_rotation(seed: int, dim: int = 3) -> np.ndarray:
    """A seeded random orthogonal matrix (for global-rotation invariance tests)."""
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((dim, dim)))
    return q * np.sign(np.diag(r))


def random_permutation(seed: int, q: int, keep_first: bool = True) -> np.ndarray:
    """A seeded relabelling of the q spin states; by default vertex 0 stays first."""
    rng = np.random.default_rng(seed)
    if keep_first:
        return np.concatenate([[0], 1 + rng.permutation(q - 1)])
    return rng.permutation(q)


def random_state(seed: int, q: int, m: int, decay: float = 0.85, signed: bool = True):
    """A seeded synthetic CTMRG state: q symmetric m x m slices P_s and a corner spectrum omega.

    omega decays geometrically from 1 (with alternating signs when `signed`), and each
    slice is a symmetric matrix with entries of order one, scaled so that max|P| = 1.
    Returns (P[q, m, m], omega[m]).
    """
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((q, m, m))
    p = 0.5 * (a + a.transpose(0, 2, 1))
    p /= np.abs(p).max()
    om = decay ** np.arange(m, dtype=np.float64)
    if signed:
        om = om * np.where(rng.random(m) < 0.2, -1.0, 1.0)
        om[0] = 1.0
    return p, om


def random_symmetric_with_spectrum(seed: int, evals: np.ndarray) -> np.ndarray:
    """Q diag(evals) Q^T with a seeded Haar-random orthogonal Q."""
    n = len(evals)
    rng = np.random.default_rng(seed)
    q, r = np.linalg.qr(rng.standard_normal((n, n)))
    q = q * np.sign(np.diag(r))
    a = (q * evals) @ q.T
    return 0.5 * (a + a.T)


def graded_spectrum(seed: int, n: int, pair_fraction: float = 0.6, ratio: float = 0.93) -> np.ndarray:
    """A graded spectrum with both signs and exact pairs, shaped like a corner-matrix spectrum."""
    rng = np.random.default_rng(seed)
    vals = []
    x = 1.0
    while len(vals) < n:
        sign = -1.0 if rng.random() < 0.25 else 1.0
        if rng.random() < pair_fraction and len(vals) + 2 <= n:
            vals += [sign * x, sign * x]
        else:
            vals.append(sign * x)
        x *= ratio
    return np.asarray(vals[:n])

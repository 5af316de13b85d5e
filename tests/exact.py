"""Exact results used to pin the oracle (test-only; independent of oracle/ and of the GPU library).

* Onsager's free energy and internal energy of the square-lattice Ising model, and
  Yang's spontaneous magnetization: textbook closed forms, evaluated with scipy
  (quadrature and the complete elliptic integral of the first kind).
* Cube model = three independent Ising copies at coupling K/3; square model = two
  copies at K/2 (the paper's Sec. I mapping): v.v' = (sum_a s_a s'_a)/n_copies.
* Tetrahedron model = four-state Potts model with K_p = 4K/3, up to the constant
  exp(-K/3) per bond; its exact critical point and the Kramers-Wannier-type duality
  of the Potts partition function.
* Brute-force partition functions of small fixed-boundary clusters of vertices,
  by direct enumeration or by an exact row-to-row contraction of the vertex network.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import integrate, special

TC_ISING = 2.0 / math.log(1.0 + math.sqrt(2.0))


def ising_minus_beta_f(K: float) -> float:
    """-beta f per site of the square-lattice Ising model (Onsager), one-dimensional integral form."""
    c2 = math.cosh(2 * K)
    k = 2.0 * math.sinh(2 * K) / (c2 * c2)

    def integrand(th):
        return math.log(0.5 * (1.0 + math.sqrt(max(0.0, 1.0 - k * k * math.sin(th) ** 2))))

    val, _ = integrate.quad(integrand, 0.0, math.pi / 2, epsabs=1e-15, epsrel=1e-15, limit=200)
    return math.log(2.0 * c2) + val / math.pi


def ising_energy(K: float) -> float:
    """Internal energy per site, u = -coth(2K) [1 + (2/pi)(2 tanh^2(2K) - 1) K1(k)]."""
    k = 2.0 * math.sinh(2 * K) / math.cosh(2 * K) ** 2
    K1 = special.ellipk(k * k)
    return -1.0 / math.tanh(2 * K) * (1.0 + 2.0 / math.pi * (2.0 * math.tanh(2 * K) ** 2 - 1.0) * K1)


def ising_magnetization(K: float) -> float:
    """Yang's spontaneous magnetization (zero above T_c)."""
    s = math.sinh(2 * K)
    if s <= 1.0:
        return 0.0
    return (1.0 - s ** -4) ** 0.125


def ising_dM_dK(K: float) -> float:
    """K-derivative of Yang's magnetization: with s = sinh 2K, M = (1 - s^-4)^(1/8) and
    dM/dK = cosh(2K) s^-5 (1 - s^-4)^(-7/8) (zero above T_c)."""
    s = math.sinh(2 * K)
    if s <= 1.0:
        return 0.0
    return math.cosh(2 * K) * s ** -5 * (1.0 - s ** -4) ** -0.875


def ising_d2F_dK2(K: float, h: float = 1e-4) -> float:
    """d^2(beta f)/dK^2 per site = -du/dK... computed by differentiating u (closed form) numerically."""
    return (ising_energy(K + h) - ising_energy(K - h)) / (2 * h)


def potts_critical_Kp(q: int) -> float:
    return math.log(1.0 + math.sqrt(q))


TC_TETRA = 4.0 / (3.0 * math.log(3.0))
TC_CUBE = TC_ISING / 3.0
TC_SQUARE = TC_ISING / 2.0


def tetra_dual_K(K: float) -> float:
    """Dual coupling of the tetrahedron model through the 4-state Potts duality (e^Kp - 1)(e^Kp* - 1) = 4."""
    v = math.exp(4.0 * K / 3.0) - 1.0
    vs = 4.0 / v
    return 0.75 * math.log(1.0 + vs)


def tetra_duality_offset(K: float) -> float:
    """-beta f_tet(K) - (-beta f_tet(K*)) predicted by duality, per site.

    Z_tet(K) = exp(-2N K/3) Z_Potts(K_p = 4K/3) (two bonds per site), and the Potts
    duality on the square lattice gives, per site, ln Z_P(v) = 2 ln v - ln q + ln Z_P(q/v)."""
    v = math.exp(4.0 * K / 3.0) - 1.0
    Ks = tetra_dual_K(K)
    return (-2.0 * K / 3.0 + 2.0 * math.log(v) - math.log(4.0)) - (-2.0 * Ks / 3.0)


# ----------------------------------------------------------------------------
# Brute-force partition functions of a 2k x 2k block of vertices
# ----------------------------------------------------------------------------
#
# The vertex lattice: vertex (r, c), 0 <= r, c < L = 2k, carries the Boltzmann weight of
# one plaquette whose four corner spins are its legs left/up/right/down; neighbouring
# vertices share a leg.  All 4L legs on the perimeter take the boundary spin s0.
# The weight of a vertex with legs (l, u, r, d) is exp(K (v_l.v_u + v_u.v_r + v_r.v_d + v_d.v_l)):
# the four bonds of the plaquette.

def _vertex_tensor(V, K):
    G = V @ V.T
    # axes (l, u, r, d)
    return np.exp(K * (G[:, :, None, None] + G[None, :, :, None] + G[None, None, :, :]
                       + G.T[:, None, None, :]))


def cluster_Z_enumerate(V, K, k, s0=0):
    """Direct sum over all internal leg configurations (tiny clusters only)."""
    V = np.asarray(V, dtype=np.float64)
    q = len(V)
    L = 2 * k
    G = V @ V.T
    # horizontal legs h[r][c] between (r, c-1) and (r, c), c = 0..L (c=0 and c=L on the boundary)
    # vertical legs  w[r][c] between (r-1, c) and (r, c), r = 0..L
    internal = []
    for r in range(L):
        for c in range(1, L):
            internal.append(("h", r, c))
    for r in range(1, L):
        for c in range(L):
            internal.append(("w", r, c))
    n = len(internal)
    total = 0.0
    for conf in itertools.product(range(q), repeat=n):
        val = dict(zip(internal, conf))

        def h(r, c):
            return s0 if c == 0 or c == L else val[("h", r, c)]

        def w(r, c):
            return s0 if r == 0 or r == L else val[("w", r, c)]

        e = 0.0
        for r in range(L):
            for c in range(L):
                l, u, rr, d = h(r, c), w(r, c), h(r, c + 1), w(r + 1, c)
                e += G[l, u] + G[u, rr] + G[rr, d] + G[d, l]
        total += math.exp(K * e)
    return total


def cluster_lnZ_transfer(V, K, k, s0=0):
    """Exact ln Z of the 2k x 2k vertex block by row-to-row contraction (no truncation).

    The state is the vector over the L vertical legs crossing a horizontal cut; a row of
    vertices is absorbed one vertex at a time.  Returns ln Z (rescaled as it goes)."""
    V = np.asarray(V, dtype=np.float64)
    q = len(V)
    L = 2 * k
    Wv = _vertex_tensor(V, K)  # (l, u, r, d)
    # state over the L vertical legs above the current row: all fixed to s0 at the top
    state = np.zeros((q,) * L)
    state[(s0,) * L] = 1.0
    lnscale = 0.0
    for r in range(L):
        # add a horizontal leg at the left boundary fixed to s0: axes (w_0..w_{L-1}, h)
        st = np.zeros(state.shape + (q,))
        st[..., s0] = state
        for c in range(L):
            # contract vertex (r, c): legs l = h (last axis), u = axis c; produce d (new axis c), r (new h)
            # st axes: (w_0 .. w_{L-1}, h); move axis c and h to the end
            st = np.moveaxis(st, c, -2)  # (..., u, l)
            # Wv axes (l, u, r, d) -> contract l and u
            st = np.tensordot(st, Wv, axes=([st.ndim - 1, st.ndim - 2], [0, 1]))  # (..., r, d)
            # put d back at position c, r as the last axis
            st = np.moveaxis(st, -1, c)
        # the right boundary leg must be s0
        state = st[..., s0]
        mx = np.abs(state).max()
        state = state / mx
        lnscale += math.log(mx)
    # the bottom legs are fixed to s0
    return lnscale + math.log(state[(s0,) * L])


# ----------------------------------------------------------------------------
# Entanglement entropy of the Ising corner (free-fermion corner transfer matrix)
# ----------------------------------------------------------------------------

def ising_ctm_epsilon(K: float) -> float:
    """Level spacing of the Ising corner transfer matrix in the ordered phase (Baxter):
    eps = pi I(k') / I(k), k = 1 / sinh^2(2K), I the complete elliptic integral of the
    first kind.  rho = C^4 / Tr C^4 is then a product of independent two-level factors
    with excitation energies 2 j eps, j = 1, 2, 3, ..."""
    k = 1.0 / math.sinh(2.0 * K) ** 2
    if k >= 1.0:
        raise ValueError("ordered phase only (T < T_c)")
    return math.pi * special.ellipk(1.0 - k * k) / special.ellipk(k * k)


def ising_ctm_entropy(K: float, levels: int = 200) -> float:
    """-Tr rho ln rho for rho = prod_j diag(1, e^{-e_j}) / (1 + e^{-e_j}), e_j = 2 j eps:
    the sum over modes of ln(1 + e^{-e_j}) + e_j / (e^{e_j} + 1)."""
    eps = ising_ctm_epsilon(K)
    s = 0.0
    for j in range(1, levels + 1):
        e = 2.0 * j * eps
        x = math.exp(-e)
        s += math.log1p(x) + e * x / (1.0 + x)
    return s


def ising_ctm_levels(K: float, count: int) -> np.ndarray:
    """The smallest `count` values of sum_j n_j e_j (n_j in {0, 1}, e_j = 2 j eps): the
    spectrum of -ln(rho / rho_max), with multiplicities (partitions into distinct parts)."""
    eps = ising_ctm_epsilon(K)
    nmax = 64
    # number of partitions of n into distinct parts, with multiplicity
    vals = []
    for n in range(nmax):
        # count partitions of n into distinct positive parts
        c = _distinct_partitions(n)
        vals.extend([2.0 * n * eps] * c)
        if len(vals) >= count:
            break
    return np.array(vals[:count])


def _distinct_partitions(n: int) -> int:
    p = [1] + [0] * n
    for part in range(1, n + 1):
        for t in range(n, part - 1, -1):
            p[t] += p[t - part]
    return p[n]


def row_transfer_bruteforce(V, K, s0, n):
    """The row-to-row transfer matrix of a straight row of n vertices with both outer
    horizontal spins fixed to s0, by direct enumeration of the row from Eqs. 1-2.

    Vertex i of the row has its horizontal spins h_{i-1} (left) and h_i (right) on
    opposite corners and its legs l_i (lower) and u_i (upper) on the other two; around
    the vertex the corners run left, lower, right, upper, and the vertex weight is
    exp(K (v_left.v_lower + v_lower.v_right + v_right.v_upper + v_upper.v_left)).
    T[(u_1..u_n), (l_1..l_n)] = sum over h_1..h_{n-1} of the product of the n weights
    (h_0 = h_n = s0), the legs in row order with u_1 / l_1 most significant."""
    V = np.asarray(V, dtype=np.float64)
    q = len(V)
    G = V @ V.T
    w = np.empty((q, q, q, q))  # w[left, lower, upper, right]
    for a in range(q):
        for b in range(q):
            for c in range(q):
                for d in range(q):
                    w[a, b, c, d] = math.exp(K * (G[a, b] + G[b, d] + G[d, c] + G[c, a]))
    # M[h][U, L]: the first i vertices with their right spin h, legs U (upper) and L (lower)
    M = np.zeros((q, 1, 1))
    M[s0, 0, 0] = 1.0
    for _ in range(n):
        R = M.shape[1]
        # new legs are the least significant: index (U, u) and (L, l)
        Mn = np.einsum("hUL,hluk->kUuLl", M, w)
        M = Mn.reshape(q, R * q, R * q)
    return M[s0]

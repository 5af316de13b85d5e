"""TEST INFRASTRUCTURE ONLY: the plain FP64 CPU oracle for the CTMRG step.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this module.  It shares no code with the GPU library and imports nothing from
it; the only code both sides use is the seeded input module (spin vectors and
random states, no arithmetic of the method).

What it computes, in the paper's order (Sec. II and Sec. III, Algorithm 3, of
Ueda, Okunishi, Yunoki and Nishino, "Corner transfer matrix renormalization
group analysis of the two-dimensional dodecahedron model"):

  * the Boltzmann vertex weight W (Eqs. 1-2) on every other plaquette;
  * the fixed ferromagnetic boundary condition through the initial P and Omega;
  * each CTMRG step: extend the corner with two half-rows and one vertex,
    diagonalize the extended corner (own Jacobi solver, jacobi.c), keep the m
    leading eigenvectors, project the extended half-row back, normalize P by its
    largest element and Omega by the fourth root of sum(omega^4) over all mq
    eigenvalues, and evaluate the entanglement entropy of Eq. 6;
  * observables at the fixed point: M (Eq. 5, from rho = C^4 / Tr C^4),
    S_E (Eq. 6), the free energy and the energy per site.

Library primitives used as single steps: numpy matmul/einsum/tensordot for the
tensor contractions, numpy sort.  No blocking, fusion or reordering beyond what
the formulas state.  The diagonalization is the oracle's own Jacobi solver by
default; eig="lapack" takes numpy's symmetric eigensolver (LAPACK) as the
single step instead, for long runs at N = q m >= 1280 where Jacobi takes
minutes per step.  Both are pinned against prescribed spectra.

Readings where the paper is silent or inconsistent (each is justified in the
design notes of the repository and pinned by the tests):

  * Leg order of W.  Eq. 1 lists the four spins of a plaquette in cyclic order.
    The extended corner C'[(alpha,s'),(beta,sigma')] contracts half-row P_s,
    the corner, half-row P_sigma and the vertex; geometrically the new spin s'
    on the row edge is adjacent to s and to sigma', and sigma' is adjacent to
    sigma.  So the weight used is
        Wt[(s,sigma),(s',sigma')] = exp(K (v_s.v_sigma + v_sigma.v_sigma'
                                           + v_sigma'.v_s' + v_s'.v_s)).
  * Coupling: K = 1/T per nearest-neighbour bond, each bond counted once
    (W on every other plaquette).
  * Eigenvalue order: descending |lambda|, ties by lambda descending, then index.
  * Truncation keeps whole multiplets: m_eff is the largest j <= min(m, dim)
    with |l_j| > rank_tol |l_1| and (j == dim or |l_j| - |l_{j+1}| > tau |l_1|).
  * Free energy: from the exact bookkeeping of the normalization factors,
    ln kappa_W = ln n_P(k) + 1/2 ln(n_C(k+1)/n_C(k)) per vertex, two sites per vertex.
  * Energy: the central plaquette energy in the environment of four corners and
    four half-rows, E = 1/2 <h_4>.
  * Convergence: Delta_k = max_j |w_j^4(k) - w_j^4(k-1)| over the kept spectrum
    (zero padded to m); the paper's |1 - S_E/S| is recorded too.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "jacobi.c")

_lib = None


def build_library(force: bool = True) -> str:
    """Compile jacobi.c into liboracle.so with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", SRC_PATH, "-o", tmp, "-lm"]
        )
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build_library(force=True)
        lib = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_jacobi.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_int]
        lib.oracle_jacobi.restype = ctypes.c_int
        lib.oracle_num_threads.argtypes = []
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ----------------------------------------------------------------------------
# Model: Eqs. 1-2
# ----------------------------------------------------------------------------

def plaquette_energy(V: np.ndarray) -> np.ndarray:
    """h4[s,sigma,s',sigma'] = -(v_s.v_sigma + v_sigma.v_sigma' + v_sigma'.v_s' + v_s'.v_s).

    Eq. 1 with J = 1; the corners of the plaquette in cyclic order are
    s, sigma, sigma', s' (the reading of the leg order described above)."""
    G = np.asarray(V, dtype=np.float64) @ np.asarray(V, dtype=np.float64).T
    # axes: (s, sigma, s', sigma')
    t1 = G[:, :, None, None]          # v_s . v_sigma
    t2 = G[None, :, None, :]          # v_sigma . v_sigma'
    t3 = G.T[None, None, :, :]        # v_sigma' . v_s'   (indexed by s', sigma')
    t4 = G.T[:, None, :, None]        # v_s' . v_s        (indexed by s, s')
    return -(t1 + t2 + t3 + t4)


def weight(V: np.ndarray, K: float) -> np.ndarray:
    """W[s,sigma,s',sigma'] = exp(-K h4) (Eq. 2, k_B = 1, K = 1/T), shape (q,q,q,q)."""
    return np.exp(-K * plaquette_energy(V))


def weight_matrix(V: np.ndarray, K: float) -> np.ndarray:
    """The q^2 x q^2 matrix Wt[(s,sigma),(s',sigma')] (row s*q+sigma, column s'*q+sigma')."""
    q = len(V)
    return weight(V, K).reshape(q * q, q * q)


# ----------------------------------------------------------------------------
# Eigensolver: Jacobi (jacobi.c)
# ----------------------------------------------------------------------------

def jacobi(A: np.ndarray, max_sweeps: int = 60):
    """Eigenvalues and eigenvectors (columns) of the symmetric matrix A, unsorted."""
    lib = _load()
    n = A.shape[0]
    a = np.array(A, dtype=np.float64, order="C", copy=True)
    ev = np.empty(n)
    vec = np.empty((n, n))
    sweeps = lib.oracle_jacobi(n, _ptr(a), _ptr(ev), _ptr(vec), max_sweeps)
    if sweeps < 0:
        raise RuntimeError("Jacobi did not converge")
    return ev, vec


def sort_spectrum(lam: np.ndarray):
    """Order: descending |lambda|, ties by lambda descending, then by index."""
    idx = np.arange(len(lam))
    return np.lexsort((idx, -lam, -np.abs(lam)))


def fix_signs(U: np.ndarray) -> np.ndarray:
    """Each column is negated if its first entry of largest magnitude is negative."""
    if U.size == 0:
        return U
    i = np.argmax(np.abs(U), axis=0)
    s = np.sign(U[i, np.arange(U.shape[1])])
    s[s == 0] = 1.0
    return U * s


def cut_dimension(lam_sorted: np.ndarray, m: int, tau: float, rank_tol: float) -> int:
    """Number of kept states: the largest j <= min(m, dim) that does not split a multiplet."""
    a = np.abs(lam_sorted)
    n = len(a)
    if n == 0 or a[0] == 0.0:
        raise ValueError("zero corner matrix")
    l1 = a[0]
    jmax = min(m, n)
    for j in range(jmax, 0, -1):
        if a[j - 1] <= rank_tol * l1:
            continue
        if j == n or a[j - 1] - a[j] > tau * l1:
            return j
    # every admissible cut splits a multiplet: keep what the rank allows
    return max(1, int(np.sum(a[:jmax] > rank_tol * l1)))


# ----------------------------------------------------------------------------
# One CTMRG step: Algorithm 3 and its Sub-CTMRG
# ----------------------------------------------------------------------------

def extend(W: np.ndarray, P: np.ndarray, omega: np.ndarray) -> np.ndarray:
    """Extended corner C' (Algorithm 3, first Sub-CTMRG call with P' = Omega P).

    X_{s sigma} = P_s Omega P_sigma (the product P^t P'),
    C'_{s' sigma'} = sum_{s,sigma} W[s,sigma,s',sigma'] X_{s sigma} (the product with w),
    returned as a (q d) x (q d) matrix with row (s', alpha) -> s'*d + alpha."""
    q, d, _ = P.shape
    X = np.einsum("sag,g,tgb->stab", P, omega, P, optimize=True)
    Cq = np.tensordot(W, X, axes=([0, 1], [0, 1]))  # (s', sigma', alpha, beta)
    return Cq.transpose(0, 2, 1, 3).reshape(q * d, q * d)


def extend_entry(W: np.ndarray, P: np.ndarray, omega: np.ndarray, row: int, col: int) -> float:
    """One entry of C' straight from the definition (for sampled checks at large sizes)."""
    q, d, _ = P.shape
    sp, a = divmod(row, d)
    tp, b = divmod(col, d)
    total = 0.0
    for s in range(q):
        for t in range(q):
            x = float(np.sum(P[s, a, :] * omega * P[t, :, b]))
            total += W[s, t, sp, tp] * x
    return total


def halfrow(W: np.ndarray, P: np.ndarray, Uk: np.ndarray) -> np.ndarray:
    """Projected extended half-row (Algorithm 3, second Sub-CTMRG call with U', then U^t X).

    U_sigma[gamma, j] = U[(sigma, gamma), j];
    Y_{s sigma} = P_s U_sigma;  Z_{s' sigma'} = sum W[s,sigma,s',sigma'] Y_{s sigma};
    Pt_{sigma'} = sum_{s'} U_{s'}^t Z_{s' sigma'}."""
    q, d, _ = P.shape
    me = Uk.shape[1]
    Us = Uk.reshape(q, d, me)
    Y = np.einsum("sag,tgj->staj", P, Us, optimize=True)
    Z = np.tensordot(W, Y, axes=([0, 1], [0, 1]))  # (s', sigma', alpha, j)
    return np.einsum("sai,staj->tij", Us, Z, optimize=True)


@dataclass
class StepResult:
    cext: np.ndarray | None
    lam: np.ndarray          # all eigenvalues of C', sorted
    U: np.ndarray            # kept eigenvectors (q d) x m_eff, sign-fixed
    m_eff: int
    n_C: float
    w: np.ndarray            # all eigenvalues / n_C
    S_E: float
    Pt: np.ndarray           # projected half-row before normalization
    n_P: float
    P: np.ndarray            # Pt / n_P
    omega: np.ndarray        # kept w
    asym: float              # max |C' - C'^T| / max |C'|


def entropy(w: np.ndarray) -> float:
    """S_E = -sum w^4 ln w^4 over all eigenvalues (Eq. 6 as written in Algorithm 3)."""
    w4 = w ** 4
    nz = w4 > 0
    return float(-np.sum(w4[nz] * np.log(w4[nz])))


def eigh(A: np.ndarray, method: str = "jacobi"):
    """Eigenvalues and eigenvectors of the symmetric A: the oracle's Jacobi solver, or
    numpy's LAPACK driver as a single library step (method="lapack")."""
    if method == "jacobi":
        return jacobi(A)
    if method == "lapack":
        return np.linalg.eigh(A)
    raise ValueError(method)


def step(W: np.ndarray, P: np.ndarray, omega: np.ndarray, m: int, tau: float = 1e-10,
         rank_tol: float = 1e-13, keep_cext: bool = False, eig: str = "jacobi") -> StepResult:
    C = extend(W, P, omega)
    amax = np.abs(C).max()
    asym = float(np.abs(C - C.T).max() / amax) if amax > 0 else 0.0
    Cs = 0.5 * (C + C.T)
    lam, vec = eigh(Cs, eig)
    order = sort_spectrum(lam)
    lam = lam[order]
    vec = vec[:, order]
    me = cut_dimension(lam, m, tau, rank_tol)
    n_C = float(np.sum(lam ** 4) ** 0.25)
    w = lam / n_C
    S_E = entropy(w)
    Uk = fix_signs(vec[:, :me])
    Pt = halfrow(W, P, Uk)
    n_P = float(np.abs(Pt).max())
    return StepResult(C if keep_cext else None, lam, Uk, me, n_C, w, S_E, Pt, n_P,
                      Pt / n_P, w[:me].copy(), asym)


# ----------------------------------------------------------------------------
# The iteration and the observables
# ----------------------------------------------------------------------------

def initial_state(q: int, bc: str = "fixed", s0: int = 0):
    """Algorithm 3 initialization: P is 1 x 1 per spin, Omega = [1].

    Fixed boundary: only the boundary spin s0 carries weight (p_11 = 1).
    Free boundary: every spin carries weight one."""
    P = np.zeros((q, 1, 1))
    if bc == "fixed":
        P[s0, 0, 0] = 1.0
    elif bc == "free":
        P[:, 0, 0] = 1.0
    else:
        raise ValueError(bc)
    return P, np.ones(1)


@dataclass
class OracleCTMRG:
    V: np.ndarray
    K: float
    m: int
    bc: str = "fixed"
    s0: int = 0
    tau: float = 1e-10
    rank_tol: float = 1e-13
    eig: str = "jacobi"
    P: np.ndarray = None
    omega: np.ndarray = None
    k: int = 0
    ln_a: float = 0.0
    ln_b: float = 0.0
    nC: list = field(default_factory=list)
    nP: list = field(default_factory=list)
    S_hist: list = field(default_factory=list)
    delta: float = float("inf")
    c_paper: float = float("inf")
    last: StepResult | None = None

    def __post_init__(self):
        self.V = np.asarray(self.V, dtype=np.float64)
        self.q = len(self.V)
        self.W = weight(self.V, self.K)
        self.H4 = plaquette_energy(self.V)
        if self.P is None:
            self.P, self.omega = initial_state(self.q, self.bc, self.s0)

    def import_state(self, P, omega, k: int = 1):
        self.P = np.array(P, dtype=np.float64)
        self.omega = np.array(omega, dtype=np.float64)
        self.k = k

    def step(self, keep_cext: bool = False) -> StepResult:
        prev = np.zeros(self.m)
        prev[: len(self.omega)] = self.omega ** 4
        r = step(self.W, self.P, self.omega, self.m, self.tau, self.rank_tol, keep_cext, self.eig)
        # bookkeeping of the true scale (P_true = a P, C_true = b Omega)
        self.ln_b = self.ln_b + 2.0 * self.ln_a + np.log(r.n_C)
        self.ln_a = self.ln_a + np.log(r.n_P)
        self.nC.append(r.n_C)
        self.nP.append(r.n_P)
        cur = np.zeros(self.m)
        cur[: r.m_eff] = r.omega ** 4
        self.delta = float(np.abs(cur - prev).max())
        S_prev = self.S_hist[-1] if self.S_hist else 0.0
        self.c_paper = abs(1.0 - r.S_E / S_prev) if S_prev != 0.0 else float("inf")
        self.S_hist.append(r.S_E)
        self.P, self.omega = r.P, r.omega
        self.k += 1
        self.last = r
        return r

    def run(self, tol: float, max_steps: int, min_steps: int = 2):
        for _ in range(max_steps):
            self.step()
            if self.k >= min_steps and self.delta < tol:
                return True
        return False

    def ln_Z(self) -> float:
        """ln Tr C_k^4 of the current (truncated) corner: 4 ln b_k + ln sum omega^4."""
        return 4.0 * self.ln_b + float(np.log(np.sum(self.omega ** 4)))

    def ln_kappa_W(self) -> float:
        """Per-vertex partition function from the normalization history (needs two steps)."""
        if len(self.nC) < 2:
            raise ValueError("needs at least two steps")
        return float(np.log(self.nP[-2]) + 0.5 * np.log(self.nC[-1] / self.nC[-2]))

    def environment_sums(self):
        """Z_b = Tr C^4, Z_h = sum_s Tr(P_s C^2 P_s C^2), Z_d = sum W Tr(C P C P C P C P)
        and the same with W replaced by W * h4, on the current state."""
        P, om, W = self.P, self.omega, self.W
        G = np.einsum("i,aij,j,bjk->abik", om, P, om, P, optimize=True)   # Omega P_a Omega P_b
        T4 = np.einsum("abik,cdki->abcd", G, G, optimize=True)           # Tr(G_ab G_cd)
        # corners of the central plaquette in cyclic order s, sigma, sigma', s'
        Zd = float(np.einsum("abcd,abdc->", W, T4))
        Zd_h = float(np.einsum("abcd,abdc->", W * self.H4, T4))
        Zb = float(np.sum(om ** 4))
        Zh = float(np.einsum("sij,j,i->", P ** 2, om ** 2, om ** 2))
        return Zb, Zh, Zd, Zd_h

    def magnetization(self) -> float:
        """Eq. 5 with rho = C'^4 / Tr C'^4 restricted to the kept eigenvectors of the last step."""
        r = self.last
        q = self.q
        d = r.U.shape[0] // q
        w4 = r.omega ** 4
        prob = np.einsum("j,sbj->s", w4, r.U.reshape(q, d, -1) ** 2) / np.sum(w4)
        if self.bc == "fixed":
            return float(prob @ (self.V @ self.V[self.s0]))
        return float(np.linalg.norm(prob @ self.V))

    def observables(self) -> dict:
        lk = self.ln_kappa_W()
        Zb, Zh, Zd, Zd_h = self.environment_sums()
        T = 1.0 / self.K
        return {
            "ln_kappa_W": lk,
            "ln_kappa_ratio": float(np.log(Zd) + np.log(Zb) - 2.0 * np.log(Zh)),
            "f": -0.5 * T * lk,
            "minus_beta_f": 0.5 * lk,
            "E": 0.5 * Zd_h / Zd,
            "M": self.magnetization(),
            "S_E": self.last.S_E,
            "m_eff": self.last.m_eff,
            "steps": self.k,
            "delta": self.delta,
            "c_paper": self.c_paper,
        }


# ----------------------------------------------------------------------------
# Effective correlation length (Sec. II, last paragraph)
# ----------------------------------------------------------------------------

def row_transfer_matrix(P: np.ndarray) -> np.ndarray:
    """The renormalized row-to-row transfer matrix T = sum_s P_s (x) P_s (d^2 x d^2).

    A full row of vertices is two half-rows, the left one P_s and its mirror image
    (equal to P_s, since W is invariant under reflection), joined at their common
    inner end spin s, which is summed.  Rows (alpha, alpha') index the upper legs of
    the left and right halves, columns (beta, beta') the lower legs."""
    q, d, _ = P.shape
    T = np.zeros((d * d, d * d))
    for s in range(q):
        T += np.kron(P[s], P[s])
    return T


def row_transfer_apply(P: np.ndarray, X: np.ndarray) -> np.ndarray:
    """T applied to a d x d matrix X (the vector of T, row-major): sum_s P_s X P_s^t."""
    return sum(P[s] @ X @ P[s].T for s in range(P.shape[0]))


def correlation_length(P: np.ndarray, method: str = "dense", count: int = 2):
    """The `count` eigenvalues of T of largest modulus (descending |lambda|, zero padded
    when T has fewer) and the effective correlation length xi_e = 1 / ln(|lambda_1| /
    |lambda_2|), in rows of vertices (0 when lambda_2 = 0).

    method "dense": all eigenvalues of T (LAPACK), for d^2 up to a few thousand;
    "arpack": the leading ones of the operator X -> sum_s P_s X P_s^t by ARPACK's
    implicitly restarted Lanczos (scipy), a single library step."""
    q, d, _ = P.shape
    if method == "dense":
        lam = np.linalg.eigvalsh(row_transfer_matrix(P))
    elif method == "arpack":
        from scipy.sparse.linalg import LinearOperator, eigsh
        op = LinearOperator((d * d, d * d), dtype=np.float64,
                            matvec=lambda x: row_transfer_apply(P, x.reshape(d, d)).ravel())
        lam = eigsh(op, k=max(count, 4), which="LM", tol=1e-14, return_eigenvectors=False)
    else:
        raise ValueError(method)
    lam = lam[np.argsort(-np.abs(lam), kind="stable")][:count]
    if lam.size < count:  # d = 1: T is 1 x 1
        lam = np.concatenate([lam, np.zeros(count - lam.size)])
    # a single state (lambda_2 = 0) correlates nothing beyond its row: xi_e = 0
    xi = 1.0 / np.log(abs(lam[0]) / abs(lam[1])) if abs(lam[1]) > 0 else 0.0
    return lam, float(xi)


def run_fixed_point(V, K, m, bc="fixed", tol=1e-12, max_steps=3000, s0=0, tau=1e-10,
                    rank_tol=1e-13, eig="jacobi"):
    o = OracleCTMRG(V, K, m, bc=bc, s0=s0, tau=tau, rank_tol=rank_tol, eig=eig)
    converged = o.run(tol, max_steps)
    obs = o.observables()
    obs["converged"] = converged
    return o, obs

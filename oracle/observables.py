"""Equal-time observables from the Green's function (oracle side).

S^i_q = <n^{Gamma^i}_q n^{Gamma^i}_{-q}> and
m^2_SO(5) = (1/(5 N^2)) sum_{i=1}^5 S^i_{q=0} (Results, SO(5)-symmetric line),
evaluated per configuration by Wick's theorem from G_ij = <c_i c_j^dagger>:
  <(c+ A c)(c+ B c)> = Tr[A(1-G)] Tr[B(1-G)] + Tr[A G B (1-G)].
"""
import numpy as np

from .model import gamma_matrices, m_matrix


def gamma_4n(gamma, n_phi):
    """One-body matrix of flavour matrix Gamma (a = 2v+s) on modes s*2N+v*N+k."""
    perm = [0, 2, 1, 3]              # (s, v) -> a = 2v + s  ordering s-major
    g = gamma[np.ix_(perm, perm)]
    return np.kron(g, np.eye(n_phi))


def structure_factor(G2n, n_phi, gamma, qx=0, qy=0):
    """S_q for one Gamma from the spin-block G (G_4N = 1 kron G)."""
    G4 = np.kron(np.eye(2), G2n)
    n4 = 4 * n_phi
    perm = [0, 2, 1, 3]
    g = gamma[np.ix_(perm, perm)]
    A = np.kron(g, m_matrix(qx, qy, n_phi))
    B = A.conj().T
    I = np.eye(n4)
    return np.trace(A @ (I - G4)) * np.trace(B @ (I - G4)) + np.trace(A @ G4 @ B @ (I - G4))


def so5_observables(G2n, n_phi):
    """Returns (S^1..S^5 at q=0, m^2_SO(5)) for one configuration."""
    s = np.array([structure_factor(G2n, n_phi, gm) for gm in gamma_matrices()])
    return s, s.real.sum() / (5.0 * n_phi * n_phi)

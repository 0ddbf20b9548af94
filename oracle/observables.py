"""Equal-time observables from the Green's function (oracle side).

S^i_q = <n^{Gamma^i}_q n^{Gamma^i}_{-q}> and
m^2_SO(5) = (1/(5 N^2)) sum_{i=1}^5 S^i_{q=0} (Results, SO(5)-symmetric line),
evaluated per configuration by Wick's theorem from G_ij = <c_i c_j^dagger>:
  <(c+ A c)(c+ B c)> = Tr[A(1-G)] Tr[B(1-G)] + Tr[A G B (1-G)].

Imaginary-time correlator (Supplementary Note 2):
  m^2_SO(5)(tau, q=0) = (1/5) sum_i <n^{Gamma^i}_{q=0}(tau) n^{Gamma^i}_{q=0}(0)>,
with, for one-body operators A at tau and B at 0 (Wick, one configuration),
  <(c+ A c)(tau) (c+ B c)(0)> = Tr[A(1-G(tau,tau))] Tr[B(1-G(0,0))]
                               - Tr[A G(tau,0) B G(0,tau)],
G(tau,0) = <c(tau) c^dagger(0)>, G(0,tau)_ij = -<c_j^dagger(tau) c_i(0)>; at
tau = 0, G(0,0^-) = -(1 - G) and the equal-time formula is recovered.
"""
import numpy as np

from .model import PAULI, form_factor, gamma_matrices, m_matrix


def gamma_4n(gamma, n_phi):
    """One-body matrix of flavour matrix Gamma (a = 2v+s) on modes s*2N+v*N+k."""
    perm = [0, 2, 1, 3]              # (s, v) -> a = 2v + s  ordering s-major
    g = gamma[np.ix_(perm, perm)]
    return np.kron(g, np.eye(n_phi))


def _orbital_density(n_phi, qx, qy, sphere):
    if sphere:
        from .sphere import density_matrix
        return density_matrix(qx, qy, n_phi)        # (l, m) on the sphere
    return m_matrix(qx, qy, n_phi)


def structure_factor(G2n, n_phi, gamma, qx=0, qy=0, sphere=False):
    """S_q for one Gamma from the spin-block G (G_4N = 1 kron G); on the
    sphere (qx, qy) is (l, m) and n_{-q} is n_{l,m}^dagger."""
    G4 = np.kron(np.eye(2), G2n)
    n4 = 4 * n_phi
    perm = [0, 2, 1, 3]
    g = gamma[np.ix_(perm, perm)]
    A = np.kron(g, _orbital_density(n_phi, qx, qy, sphere))
    B = A.conj().T
    I = np.eye(n4)
    return np.trace(A @ (I - G4)) * np.trace(B @ (I - G4)) + np.trace(A @ G4 @ B @ (I - G4))


def so5_observables(G2n, n_phi, sphere=False):
    """Returns (S^1..S^5 at q=0 (l = m = 0 on the sphere), m^2_SO(5)) for one configuration."""
    s = np.array([structure_factor(G2n, n_phi, gm, sphere=sphere) for gm in gamma_matrices()])
    return s, s.real.sum() / (5.0 * n_phi * n_phi)


def _density_4n(gamma, n_phi, qx=0, qy=0, sphere=False):
    perm = [0, 2, 1, 3]
    g = gamma[np.ix_(perm, perm)]
    return np.kron(g, _orbital_density(n_phi, qx, qy, sphere))


def so5_correlator(Gt0, G0t, Gtt, G00, n_phi, sphere=False):
    """<n^{Gamma^i}_{q=0}(tau) n^{Gamma^i}_{q=0}(0)> for i = 1..5 (complex, one
    configuration) and their mean m^2_SO(5)(tau, q=0), from the spin-block
    Green's functions G(tau,0), G(0,tau), G(tau,tau) and G(0,0)."""
    E = np.eye(2)
    Xt0, X0t = np.kron(E, Gt0), np.kron(E, G0t)
    Xtt, X00 = np.kron(E, Gtt), np.kron(E, G00)
    I = np.eye(4 * n_phi)
    c = []
    for gm in gamma_matrices():
        A = _density_4n(gm, n_phi, sphere=sphere)
        B = A.conj().T                     # n_{-q} at q = 0
        c.append(np.trace(A @ (I - Xtt)) * np.trace(B @ (I - X00)) - np.trace(A @ Xt0 @ B @ X0t))
    c = np.array(c)
    return c, c.sum() / 5.0


def _background(qx, qy, n_phi):
    """c-number of the O^0 density operator (eq. torus density operator): -2 per
    orbital at q_y = 0 (mod N), summed with the operator's phases."""
    if qy % n_phi:
        return 0.0
    f = form_factor(qx, qy, n_phi)
    return 2.0 * sum(f * np.exp(1j * np.pi * (2 * k - qy) * qx / n_phi) for k in range(1, n_phi + 1))


def fierz_energy(G2n, n_phi, qs, g):
    """<H> of one configuration for H = sum_i g_i sum_q n^{O^i}_q n^{O^i}_{-q}
    (eq. newmodel, O^i = tau^i (x) 1_spin, i = 0..3; the O^0 operator carries its
    background), by Wick's theorem from the spin-block G (torus). With
    n = c+ A c - b: <n_q n_{-q}> = Tr[A(1-G)] Tr[B(1-G)] + Tr[A G B (1-G)]
    - b_{-q} Tr[A(1-G)] - b_q Tr[B(1-G)] + b_q b_{-q}.
    G2n: one n x n matrix, or a stack [..., n, n] (one energy per matrix)."""
    G2n = np.asarray(G2n)
    n2 = 2 * n_phi
    G4 = np.zeros(G2n.shape[:-2] + (2 * n2, 2 * n2), dtype=complex)
    G4[..., :n2, :n2] = G2n                 # G_4N = 1_spin (x) G
    G4[..., n2:, n2:] = G2n
    IG = np.eye(2 * n2) - G4
    e = np.zeros(G2n.shape[:-2], dtype=complex)
    for i in range(4):
        gamma = np.kron(PAULI[i], PAULI[0])
        for qx, qy in qs:
            A = _density_4n(gamma, n_phi, qx, qy)
            B = _density_4n(gamma, n_phi, -qx, -qy)
            tA = np.einsum("xy,...yx->...", A, IG)
            tB = np.einsum("xy,...yx->...", B, IG)
            w = tA * tB + np.einsum("...xz,...zx->...", A @ G4, B @ IG)
            if i == 0:
                bA, bB = _background(qx, qy, n_phi), _background(-qx, -qy, n_phi)
                w = w + bA * bB - bB * tA - bA * tB
            e = e + g[i] * w
    return e

"""Second-quantised construction in Fock space (oracle side, tiny sizes).

Builds the density operators of the torus regularisation directly from the
printed formula (Methods, "Toric regularization", eq. torus density operator)
with Jordan-Wigner fermions, and the Hamiltonians before and after the Fierz
rewrite (eqs. model and newmodel). Used to pin the one-body tables of
model.py (Fock-trace identity), the Hubbard-Stratonovich identity (eq. HS
transform) and the observables, and for exact diagonalisation at N = 2.

Mode index of the 4N fermions: x = s*2N + v*N + (k-1), flavour a = 2v + s
(Gamma = tau kron sigma, valley outer).
"""
import numpy as np

from .model import form_factor, gamma_matrices, PAULI


def annihilators(n_modes):
    """Dense Jordan-Wigner annihilation operators c_x on 2^n_modes states."""
    a = np.array([[0.0, 1.0], [0.0, 0.0]])     # |0><1| on one mode
    z = np.diag([1.0, -1.0])
    eye = np.eye(2)
    ops = []
    for x in range(n_modes):
        m = np.array([[1.0]])
        for y in range(n_modes):
            f = z if y < x else (a if y == x else eye)
            m = np.kron(m, f)
        ops.append(m)
    return ops


def mode(n_phi, k, a):
    """Fock mode of orbital k (1-based) and flavour a = 2v + s."""
    v, s = a // 2, a % 2
    return s * 2 * n_phi + v * n_phi + (k - 1)


def density_operator(cs, n_phi, qx, qy, gamma, background):
    """n^Gamma_q (eq. torus density operator): F(q) sum_k sum_ab
    exp(i pi (2k - qy) qx / N) (c+_{k,a} Gamma_ab c_{k-qy,b} - background),
    with the background -2 per orbital for Gamma^0 and qy = 0 (mod N)."""
    n = n_phi
    dim = cs[0].shape[0]
    f = form_factor(qx, qy, n)
    out = np.zeros((dim, dim), dtype=complex)
    for k in range(1, n + 1):
        ph = f * np.exp(1j * np.pi * (2 * k - qy) * qx / n)
        kk = ((k - qy - 1) % n) + 1
        for a in range(4):
            for b in range(4):
                if gamma[a, b] != 0:
                    out += ph * gamma[a, b] * (cs[mode(n, k, a)].T @ cs[mode(n, kk, b)])
        if background and (qy % n) == 0:
            out -= 2.0 * ph * np.eye(dim)
    return out


def component_operators(cs, n_phi, comps, o2, background):
    """Hermitian HS components of one Fierz channel O = o2 kron 1_spin built
    from the density operators (sum-of-squares equation)."""
    gamma = np.kron(o2, PAULI[0])
    out = []
    for kind, qx, qy in comps:
        nq = density_operator(cs, n_phi, qx, qy, gamma, background)
        if kind == 'S':
            out.append(np.sqrt(2.0) * nq)
        else:
            nmq = nq.conj().T
            out.append(nq + nmq if kind == 'A' else 1j * (nq - nmq))
    return out


def hamiltonian_fierz(cs, n_phi, qs, g):
    """H = sum_i g_i sum_q n^{O^i}_q n^{O^i}_{-q} (eq. newmodel), with n_{-q}
    built from the formula at -q."""
    dim = cs[0].shape[0]
    H = np.zeros((dim, dim), dtype=complex)
    for i in range(4):
        gamma = np.kron(PAULI[i], PAULI[0])
        for (qx, qy) in qs:
            a = density_operator(cs, n_phi, qx, qy, gamma, i == 0)
            b = density_operator(cs, n_phi, -qx, -qy, gamma, i == 0)
            H += g[i] * (a @ b)
    return H


def hamiltonian_original(cs, n_phi, qs, u0, uk, un):
    """H = U0 H_0 - sum_{i=1}^5 U_i H_i with H_i = sum_q n^{Gamma^i}_q n^{Gamma^i}_{-q}
    (eq. model), U_1 = U_2 = U_K, U_3 = U_4 = U_5 = U_N."""
    dim = cs[0].shape[0]
    H = np.zeros((dim, dim), dtype=complex)
    gam = [np.eye(4, dtype=complex)] + gamma_matrices()
    coef = [u0, -uk, -uk, -un, -un, -un]
    for i in range(6):
        for (qx, qy) in qs:
            a = density_operator(cs, n_phi, qx, qy, gam[i], i == 0)
            b = density_operator(cs, n_phi, -qx, -qy, gam[i], i == 0)
            H += coef[i] * (a @ b)
    return H


def bilinear(cs, M):
    """Fock operator c^dagger M c of a one-body matrix M on the modes."""
    dim = cs[0].shape[0]
    out = np.zeros((dim, dim), dtype=complex)
    nz = np.argwhere(M != 0)
    for x, y in nz:
        out += M[x, y] * (cs[x].T @ cs[y])
    return out


def density_operator_sphere(cs, n_phi, l, m, gamma, background):
    """n^Gamma_{l,m} on the sphere (eq. sphere density operator): sum over
    orbitals k and flavours a, b of the 3j weight times (c+_{k,a} Gamma_ab
    c_{k',b} - background), m_{k'} = m_k + m, background -2 per orbital for
    Gamma^0 and m = 0."""
    from .sphere import density_matrix
    W = density_matrix(l, m, n_phi)
    dim = cs[0].shape[0]
    out = np.zeros((dim, dim), dtype=complex)
    for r, c in np.argwhere(W != 0):
        for a in range(4):
            for b in range(4):
                if gamma[a, b] != 0:
                    out += W[r, c] * gamma[a, b] * (cs[mode(n_phi, r + 1, a)].T @ cs[mode(n_phi, c + 1, b)])
        if background and m == 0 and r == c:
            out -= 2.0 * W[r, c] * np.eye(dim)
    return out


def component_operators_sphere(cs, n_phi, comps, o2, background):
    """Hermitian HS components of one Fierz channel on the sphere:
    sqrt(2) n_{l,0}, n_{l,m} + n_{l,m}^+, i (n_{l,m} - n_{l,m}^+)."""
    gamma = np.kron(o2, PAULI[0])
    out = []
    for kind, l, m in comps:
        nq = density_operator_sphere(cs, n_phi, l, m, gamma, background)
        if kind == 'S':
            out.append(np.sqrt(2.0) * nq)
        else:
            nmq = nq.conj().T
            out.append(nq + nmq if kind == 'A' else 1j * (nq - nmq))
    return out


def hamiltonian_sphere(cs, n_phi, coef, gammas, background_first):
    """sum_i coef_i sum_{l,m} n^{G_i}_{l,m} (n^{G_i}_{l,m})^+ over every (l, m),
    l <= 2s (the sphere's pair n_q n_{-q})."""
    from .sphere import momenta
    dim = cs[0].shape[0]
    H = np.zeros((dim, dim), dtype=complex)
    for i, gm in enumerate(gammas):
        for (l, m) in momenta(n_phi):
            a = density_operator_sphere(cs, n_phi, l, m, gm, background_first and i == 0)
            H += coef[i] * (a @ a.conj().T)
    return H


def thermal_expectation(H, O, beta):
    """Tr[e^{-beta H} O] / Tr[e^{-beta H}] by exact diagonalisation of the
    Hermitian Fock-space Hamiltonian H (all particle numbers, as the
    determinant weight of the auxiliary-field method)."""
    ev, V = np.linalg.eigh(H)
    w = np.exp(-beta * (ev - ev.min()))
    ov = np.einsum("ij,jk,ki->i", V.conj().T, O, V)
    return float(np.real(np.sum(w * ov) / np.sum(w)))

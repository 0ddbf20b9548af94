"""Model tables of the torus-regularised projected SO(5) model (oracle side).

Follows the paper's Methods: "Toric regularization" (LLL basis, momentum grid,
density operator with Gaussian form factor and background term), "Interaction
decoupling via Fierz identity" (channels O^0..O^3 and couplings g_0..g_3) and
"Continuous Hubbard-Stratonovich transformation" (sum of squares, alpha).

Conventions (readings, see the design notes):
  * orbital k runs 1..N in the phase of the density operator, the orbital
    shift k - q_y is taken modulo N (torus); matrices use 0-based rows.
  * the background term is -2 per orbital for the O^0 channel and for
    q_y = 0 (mod N); as a c-number it equals -2 tr(m_q).
  * one real HS component per Hermitian square: sqrt(2) n_0 for q = 0 (and for
    the other self-conjugate momenta of the Brillouin-zone mode),
    n_q + n_{-q} and i(n_q - n_{-q}) for each q of the half set.
  * spin-block index v*N + k (valley major); the full 4N index is
    s*2N + v*N + k.
"""
import numpy as np

# q-set modes
Q_PAPER = 0      # all integer (qx,qy) with exp(-2 pi |q|^2/(4N)) > 0.01
Q_RADIUS = 1     # |q| l_B <= q_max
Q_BZ = 2         # the N^2 momenta modulo N, representatives in (-N/2, N/2]
Q_LIST = 3       # explicit list, closed under q -> -q
Q_SPHERE = 4     # spherical regularisation: every (l, m), l <= 2s (oracle/sphere.py)

PAULI = {
    0: np.eye(2, dtype=complex),
    1: np.array([[0, 1], [1, 0]], dtype=complex),
    2: np.array([[0, -1j], [1j, 0]], dtype=complex),
    3: np.array([[1, 0], [0, -1]], dtype=complex),
}


def form_factor(qx, qy, n_phi):
    """Gaussian LLL form factor of the torus density operator (eq. torus
    density operator): exp(-2 pi (qx^2+qy^2)/(4N)) / (4 pi sqrt(N))."""
    return np.exp(-2.0 * np.pi * (qx * qx + qy * qy) / (4.0 * n_phi)) / (4.0 * np.pi * np.sqrt(n_phi))


def m_matrix(qx, qy, n_phi):
    """Orbital matrix of the torus density operator for momentum (qx, qy):
    (m_q)[k, k'] = F(q) exp(i pi (2k - qy) qx / N) if k' = k - qy (mod N),
    with k = 1..N (eq. torus density operator)."""
    n = n_phi
    m = np.zeros((n, n), dtype=complex)
    f = form_factor(qx, qy, n)
    for r in range(n):
        k = r + 1
        col = (r - qy) % n
        m[r, col] += f * np.exp(1j * np.pi * (2 * k - qy) * qx / n)
    return m


def _bz_range(n_phi):
    lo = -(n_phi // 2) + (1 if n_phi % 2 == 0 else 0)
    hi = n_phi // 2
    return range(lo, hi + 1)


def momentum_set(n_phi, q_mode=Q_PAPER, q_max=None, q_list=None):
    """Full momentum set of the model (Toric regularization: cutoff on the
    form factor; other modes are readings for the configured workloads)."""
    n = n_phi
    if q_mode == Q_PAPER:
        r = int(np.ceil(np.sqrt(4.0 * n * np.log(100.0) / (2.0 * np.pi)))) + 1
        qs = [(qx, qy) for qy in range(-r, r + 1) for qx in range(-r, r + 1)
              if np.exp(-2.0 * np.pi * (qx * qx + qy * qy) / (4.0 * n)) > 0.01]
    elif q_mode == Q_RADIUS:
        r = int(np.ceil(q_max * np.sqrt(n / (2.0 * np.pi)))) + 1
        qs = [(qx, qy) for qy in range(-r, r + 1) for qx in range(-r, r + 1)
              if (2.0 * np.pi / n) * (qx * qx + qy * qy) <= q_max * q_max * (1 + 1e-12)]
    elif q_mode == Q_BZ:
        qs = [(qx, qy) for qy in _bz_range(n) for qx in _bz_range(n)]
    elif q_mode == Q_LIST:
        qs = [tuple(int(v) for v in q) for q in q_list]
        s = set(qs)
        if len(s) != len(qs) or any((-a, -b) not in s for a, b in qs):
            raise ValueError("explicit q list must be distinct and closed under q -> -q")
    else:
        raise ValueError("unknown q mode")
    return qs


def _wrap_bz(v, n):
    r = v % n
    hi = n // 2
    return r - n if r > hi else r


def components(n_phi, q_mode=Q_PAPER, q_max=None, q_list=None):
    """Real HS components of one channel (sum-of-squares equation).

    Returns a list of (kind, qx, qy) with kind in {'S', 'A', 'C'}:
    'S' -> sqrt(2) m_q (self-conjugate q), 'A' -> m_q + m_q^dagger,
    'C' -> i (m_q - m_q^dagger). Component 0 is q = 0; the rest follow the
    canonical half set sorted by (qy, qx).
    """
    n = n_phi
    qs = momentum_set(n, q_mode, q_max, q_list)
    items = []
    if q_mode == Q_BZ:
        for (qx, qy) in qs:
            if (qx, qy) == (0, 0):
                continue
            px, py = _wrap_bz(-qx, n), _wrap_bz(-qy, n)
            if (px, py) == (qx, qy):
                items.append(('S', qx, qy))
            elif (qy, qx) > (py, px):
                items.append(('P', qx, qy))
    else:
        for (qx, qy) in qs:
            if qy > 0 or (qy == 0 and qx > 0):
                items.append(('P', qx, qy))
    items.sort(key=lambda t: (t[2], t[1]))
    comps = [('S', 0, 0)] if (0, 0) in qs else []
    for kind, qx, qy in items:
        if kind == 'S':
            comps.append(('S', qx, qy))
        else:
            comps.append(('A', qx, qy))
            comps.append(('C', qx, qy))
    return comps


def component_matrix(kind, qx, qy, n_phi):
    m = m_matrix(qx, qy, n_phi)
    if kind == 'S':
        return np.sqrt(2.0) * m
    if kind == 'A':
        return m + m.conj().T
    if kind == 'C':
        return 1j * (m - m.conj().T)
    raise ValueError(kind)


def channel_table(u0, uk, un, dtau):
    """Fierz channels (eq. newmodel) and HS couplings (eq. HS transform):
    o_i in {1, tau_x, tau_y, tau_z}, g = (U0+UN, -(UK+UN), -(UK+UN), 2UN),
    alpha_i = sqrt(-dtau g_i) on the principal branch."""
    g = np.array([u0 + un, -(uk + un), -(uk + un), 2.0 * un], dtype=float)
    alpha = np.sqrt((-dtau * g).astype(complex))
    o = np.stack([PAULI[0], PAULI[1], PAULI[2], PAULI[3]])
    return o, g, alpha


class Model:
    """All tables of one model instance (FP64, host side)."""

    def __init__(self, n_phi, l_tau, dtau, u0=1.0, uk=0.0, un=0.0,
                 q_mode=Q_PAPER, q_max=None, q_list=None):
        self.n_phi = int(n_phi)
        self.l_tau = int(l_tau)
        self.dtau = float(dtau)
        self.u0, self.uk, self.un = float(u0), float(uk), float(un)
        self.sphere = q_mode == Q_SPHERE
        if self.sphere:
            from . import sphere
            self.comps = sphere.components(n_phi)
            self.qmats = np.stack([sphere.component_matrix(k, l, m, n_phi) for (k, l, m) in self.comps])
        else:
            self.comps = components(n_phi, q_mode, q_max, q_list)
            self.qmats = np.stack([component_matrix(k, qx, qy, n_phi) for (k, qx, qy) in self.comps])
        self.n_q = len(self.comps)
        # background c-number of each component: -2 tr(q_c) (density operator)
        self.beta = np.array([-2.0 * np.trace(q) for q in self.qmats])
        self.o, self.g, self.alpha = channel_table(u0, uk, un, dtau)
        self.n = 2 * self.n_phi

    def h(self, phi_ci):
        """h = sum_c phi_c q_c for one channel's components."""
        return np.tensordot(phi_ci, self.qmats, axes=(0, 0))

    def V(self, phi_tau, i):
        """One-body exponent of channel i on the spin block:
        alpha_i * (o_i kron h_i) (HS transform, Fierz channel O^i)."""
        return self.alpha[i] * np.kron(self.o[i], self.h(phi_tau[i]))

    def c_tau(self, phi_tau):
        """Background c-number of slice tau: alpha_0 sum_c phi^0_c beta_c."""
        return self.alpha[0] * np.dot(phi_tau[0], self.beta)


def gamma_matrices():
    """Gamma^1..Gamma^5 (Results, model section) in flavour space a = 2v + s:
    tau_x x 1, tau_y x 1, tau_z x sigma_x, tau_z x sigma_y, tau_z x sigma_z."""
    t, s = PAULI, PAULI
    return [np.kron(t[1], s[0]), np.kron(t[2], s[0]), np.kron(t[3], s[1]),
            np.kron(t[3], s[2]), np.kron(t[3], s[3])]


def su4_generators():
    """T^1..T^16 = tau^a kron sigma^b in the paper's order (Fierz section)."""
    return [np.kron(PAULI[a], PAULI[b]) for a in range(4) for b in range(4)]

"""Continuous-field DQMC quantities and the MALA sweep (oracle side, FP64).

Per-configuration quantities are their plain definitions (Methods,
"Continuous Hubbard-Stratonovich transformation"):
  B_tau = exp(V_0) exp(V_1) exp(V_2) exp(V_3),  V_i = alpha_i o_i kron h_i
  B(tau2, tau1) = B_tau2 ... B_{tau1+1}
  w(phi) = exp(-S_0) exp(sum_tau c_tau) det(1 + B(beta,0))^2   (two spins)
  G(tau) = (1 + B(tau,0) B(beta,tau))^{-1}     (eq. green function)
  G(tau,0) = B(tau,0) G(0),  G(0,tau) = -(1 - G(0)) B(tau,0)^{-1}
                                               (time-displaced, Suppl. Note 2)
computed with dense products, inverses and LAPACK determinants.

The Markov chain follows the Methods section "Langevin-based global update
scheme": one Langevin proposal for all fields of a slice (eq. Langevin
proposal), the Metropolis-Hastings test with the proposal density, and the
adaptive step size after every sweep. The drift is the gradient of the
action with the derivative of each channel exponential taken to first order
(the printed gradient formula is garbled; any deterministic drift keeps the
chain exact). The exact gradient (Frechet derivative of exp) is provided for
the pins.

Slices are visited tau = 1..L; the noise of slice tau is eta (4 n_q normals,
channel-major) and u, read from a replay buffer.
"""
import numpy as np
import scipy.linalg as sla

from .model import Model


def slice_exps(model: Model, phi_tau):
    """Channel exponentials exp(V_i) and exp(-V_i) of one slice."""
    E, Einv = [], []
    for i in range(4):
        V = model.V(phi_tau, i)
        E.append(sla.expm(V))
        Einv.append(sla.expm(-V))
    return E, Einv


def b_slice(model: Model, phi_tau, exps=None):
    """Slice propagator B_tau = E_0 E_1 E_2 E_3 (one field set per channel)."""
    E, _ = exps if exps is not None else slice_exps(model, phi_tau)
    return E[0] @ E[1] @ E[2] @ E[3]


def propagators(model: Model, phi):
    return [b_slice(model, phi[t]) for t in range(model.l_tau)]


def b_range(Bs, t2, t1, n):
    """B(t2, t1) = B_{t2} ... B_{t1+1} (slices are 1-based: Bs[t-1] = B_t)."""
    out = np.eye(n, dtype=complex)
    for t in range(t1 + 1, t2 + 1):
        out = Bs[t - 1] @ out
    return out


def green(model: Model, phi, tau, Bs=None):
    """G(tau) = (1 + B(tau,0) B(beta,tau))^{-1} on the spin block (n = 2N)."""
    n, L = model.n, model.l_tau
    if Bs is None:
        Bs = propagators(model, phi)
    A = b_range(Bs, tau, 0, n) @ b_range(Bs, L, tau, n)
    return np.linalg.inv(np.eye(n) + A)


def b_range_inv(model: Model, phi, t2, t1):
    """B(t2, t1)^{-1} = B_{t1+1}^{-1} ... B_{t2}^{-1}, each slice inverse the
    product of the channel exponentials exp(-V_i) in reverse order."""
    n = model.n
    out = np.eye(n, dtype=complex)
    for t in range(t1 + 1, t2 + 1):
        _, Einv = slice_exps(model, phi[t - 1])
        out = out @ (Einv[3] @ Einv[2] @ Einv[1] @ Einv[0])
    return out


def green_displaced(model: Model, phi, tau, Bs=None):
    """Time-displaced Green's functions of one configuration, 0 <= tau <= L
    (spin block), from their definitions with G(0) = (1 + B(beta,0))^{-1}:
      G(tau,0) = <c(tau) c^dagger(0)>           = B(tau,0) G(0)
      G(0,tau) = -<c^dagger(tau) c(0)> (as [i,j]: -<c_j^dagger(tau) c_i(0)>)
               = -(1 - G(0)) B(tau,0)^{-1}
      G(tau,tau) = (1 + B(tau,0) B(beta,tau))^{-1}
    The imaginary-time correlator of the SO(5) order parameter (Supplementary
    Note 2) is built from these by Wick's theorem. Returns the three."""
    n, L = model.n, model.l_tau
    if Bs is None:
        Bs = propagators(model, phi)
    G0 = green(model, phi, 0, Bs)
    Gt0 = b_range(Bs, tau, 0, n) @ G0
    G0t = -(np.eye(n) - G0) @ b_range_inv(model, phi, tau, 0)
    Gtt = green(model, phi, tau, Bs)
    return Gt0, G0t, Gtt


def green_4n(G):
    """Full 4N Green's function 1_spin kron G (spin decouples after Fierz)."""
    return np.kron(np.eye(2), G)


def logdet(model: Model, phi, Bs=None):
    """ln of the fermion weight: sum_tau c_tau + 2 ln det(1 + B(beta,0))
    (complex; real up to 2 pi i for the sign-free model)."""
    n, L = model.n, model.l_tau
    if Bs is None:
        Bs = propagators(model, phi)
    sgn, ld = np.linalg.slogdet(np.eye(n) + b_range(Bs, L, 0, n))
    c = sum(model.c_tau(phi[t]) for t in range(L))
    return c + 2.0 * (ld + np.log(sgn))


def _channel_frames(model: Model, phi_tau, G, exps=None):
    """G_i = (E_0 ... E_{i-1})^{-1} G (E_0 ... E_{i-1}) for i = 0..3:
    the equal-time G moved to the position of channel i inside the slice."""
    E, Einv = exps if exps is not None else slice_exps(model, phi_tau)
    out = [G]
    for i in range(1, 4):
        out.append(Einv[i - 1] @ out[-1] @ E[i - 1])
    return out


def channel_traces(model: Model, Gi):
    """t^i_c = alpha_i Tr[(1 - G_i)(o_i kron q_c)] for all channels and components."""
    n, N = model.n, model.n_phi
    t = np.empty((4, model.n_q), dtype=complex)
    for i in range(4):
        Z = np.eye(n) - Gi[i]
        # Tr[Z (o kron q)] = sum_{v,v'} o[v',v] Tr[Z^{v v'} q]   (Kronecker identity)
        Y = sum(model.o[i][vp, v] * Z[v * N:(v + 1) * N, vp * N:(vp + 1) * N]
                for v in range(2) for vp in range(2))
        t[i] = model.alpha[i] * np.einsum('ckj,jk->c', model.qmats, Y)
    return t


def drift(model: Model, phi_tau, G, exps=None):
    """D = -dS/dphi for slice tau with each channel exponential differentiated to
    first order: D^i_c = -phi^i_c + 2 Re t^i_c (factor 2: two spins)."""
    t = channel_traces(model, _channel_frames(model, phi_tau, G, exps))
    return -phi_tau + 2.0 * t.real


def exact_grad_lnw(model: Model, phi, tau):
    """d ln w / d phi^i_{tau,c} by Jacobi's formula with the exact Frechet
    derivative of each channel exponential:
      2 Tr[(1 - G(tau)) dB_tau B_tau^{-1}] + alpha_0 beta_c delta_{i0}."""
    n = model.n
    Bs = propagators(model, phi)
    G = green(model, phi, tau, Bs)
    ph = phi[tau - 1]
    E, Einv = slice_exps(model, ph)
    Binv = Einv[3] @ Einv[2] @ Einv[1] @ Einv[0]
    out = np.empty((4, model.n_q), dtype=complex)
    for i in range(4):
        V = model.V(ph, i)
        left = np.eye(n, dtype=complex)
        for j in range(i):
            left = left @ E[j]
        right = np.eye(n, dtype=complex)
        for j in range(i + 1, 4):
            right = right @ E[j]
        for c in range(model.n_q):
            dV = model.alpha[i] * np.kron(model.o[i], model.qmats[c])
            _, L = sla.expm_frechet(V, dV)
            dB = left @ L @ right
            out[i, c] = 2.0 * np.trace((np.eye(n) - G) @ dB @ Binv)
    out[0] += model.alpha[0] * model.beta
    return out


class Chain:
    """One Markov chain of the CF-DQMC sweep (Methods, Langevin-based global
    update scheme), run in the paper's order on plain definitions."""

    def __init__(self, model: Model, phi, eps0=0.5, r0=0.574, deps=0.1,
                 eps_min=1e-3, eps_max=5.0, adapt=True):
        self.m = model
        self.phi = np.array(phi, dtype=float).copy()
        self.eps = float(eps0)
        self.r0, self.deps = float(r0), float(deps)
        self.eps_min, self.eps_max = float(eps_min), float(eps_max)
        self.adapt = bool(adapt)
        self.history = []          # per slice: (sweep, tau, lnA, accepted)
        self.phase_err = 0.0

    def sweep(self, replay, max_slices=None):
        """One sweep tau = 1..L (or the first max_slices slices, for timing
        samples). replay: [L][4 n_q + 1] (eta..., u)."""
        m = self.m
        n, L, nq = m.n, m.l_tau, m.n_q
        I = np.eye(n)
        X = [slice_exps(m, self.phi[t]) for t in range(L)]
        Bs = [b_slice(m, None, X[t]) for t in range(L)]
        # suffix products B(beta, tau) of the slices not yet visited
        S = [None] * (L + 1)
        S[L] = np.eye(n, dtype=complex)
        for t in range(L, 0, -1):
            S[t - 1] = S[t] @ Bs[t - 1]
        P = np.eye(n, dtype=complex)          # B(tau-1, 0) of the updated slices
        acc = 0
        eps = self.eps
        for t in range(1, L + 1):
            if max_slices is not None and t > max_slices:
                return acc
            ph = self.phi[t - 1]
            A = Bs[t - 1] @ P @ S[t]
            G = np.linalg.inv(I + A)
            D = drift(m, ph, G, X[t - 1])
            eta = replay[t - 1, :4 * nq].reshape(4, nq)
            u = replay[t - 1, 4 * nq]
            php = ph + 0.5 * eps * eps * D + eps * eta
            Xp = slice_exps(m, php)
            Bp = b_slice(m, None, Xp)
            Ap = Bp @ P @ S[t]
            s0, l0 = np.linalg.slogdet(I + A)
            s1, l1 = np.linalg.slogdet(I + Ap)
            dlnw = (m.c_tau(php) - m.c_tau(ph)) + 2.0 * ((l1 + np.log(s1)) - (l0 + np.log(s0)))
            ph_im = np.angle(np.exp(1j * dlnw.imag))
            self.phase_err = max(self.phase_err, abs(ph_im))
            Gp = np.linalg.inv(I + Ap)
            Dp = drift(m, php, Gp, Xp)
            ln_q_fwd = -np.sum((php - ph - 0.5 * eps * eps * D) ** 2) / (2 * eps * eps)
            ln_q_rev = -np.sum((ph - php - 0.5 * eps * eps * Dp) ** 2) / (2 * eps * eps)
            lnA = -0.5 * (np.sum(php ** 2) - np.sum(ph ** 2)) + dlnw.real + ln_q_rev - ln_q_fwd
            accepted = bool(np.log(u) < lnA) if u > 0 else True
            self.history.append((t, lnA, accepted))
            if accepted:
                acc += 1
                self.phi[t - 1] = php
                Bs[t - 1] = Bp
                X[t - 1] = Xp
            P = Bs[t - 1] @ P
        if self.adapt:
            r_a = acc / L
            self.eps = min(max(self.eps + (r_a - self.r0) * self.deps, self.eps_min), self.eps_max)
        return acc

    def run(self, replay_sweeps):
        return [self.sweep(r) for r in replay_sweeps]

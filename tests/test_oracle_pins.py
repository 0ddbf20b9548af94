"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test names the passage it checks. None of them compares the oracle with
itself: Fock-space constructions are built from the printed second-quantised
formulas, closed forms are derived by hand, brute force uses mpmath at high
precision, and gradients are checked by finite differences.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import dqmc, fock
from oracle.model import (Model, PAULI, Q_BZ, Q_PAPER, Q_RADIUS, components,
                          form_factor, m_matrix, su4_generators)
from oracle.observables import fierz_energy, so5_observables, structure_factor


# ---------------------------------------------------------------- model tables

@pytest.mark.parametrize("n_phi,expect", [(6, 57), (24, 221), (36, 333), (48, 437),
                                          (72, 665), (100, 933), (140, 1305)])
def test_paper_cutoff_counts(n_phi, expect):
    """Toric regularization: momenta with exp(-2 pi |q|^2/(4N)) > 0.01; the count
    grows ~ N (the paper states N_q proportional to N_phi on the torus)."""
    assert len(components(n_phi, Q_PAPER)) == expect


def test_radius_and_bz_counts():
    assert len(components(36, Q_RADIUS, 3.0)) == 161
    for n in (4, 5, 6, 8):
        assert len(components(n, Q_BZ)) == n * n


@pytest.mark.parametrize("qx,qy", [(1, 0), (2, 3), (-1, 2), (3, -2)])
def test_density_matrix_adjoint(qx, qy):
    """n_q^dagger = n_{-q} for the torus density operator."""
    n = 7
    assert np.abs(m_matrix(qx, qy, n).conj().T - m_matrix(-qx, -qy, n)).max() < 1e-15


def test_components_hermitian():
    for mode in (Q_PAPER, Q_BZ):
        m = Model(6, 2, 0.1, q_mode=mode)
        for q in m.qmats:
            assert np.abs(q - q.conj().T).max() < 1e-15


# ---------------------------------------------------------------- Fierz identity

def test_fierz_single_orbital_exact():
    """Eq. fieq on one orbital (16-dim Fock space of 4 flavours):
    -(T14)^2-(T15)^2-(T16)^2 = (T1-2)^2-(T5)^2-(T9)^2+2(T13)^2-4, with
    (X) = c^dagger X c; and the Gamma identification Gamma^0..5 = T1,T5,T9,T14,T15,T16."""
    cs = fock.annihilators(4)
    T = su4_generators()

    def op(M):
        out = np.zeros((16, 16), dtype=complex)
        for a in range(4):
            for b in range(4):
                out += M[a, b] * (cs[a].T @ cs[b])
        return out
    O = {i: op(T[i - 1]) for i in (1, 5, 9, 13, 14, 15, 16)}
    I = np.eye(16)
    lhs = -(O[14] @ O[14]) - O[15] @ O[15] - O[16] @ O[16]
    rhs = (O[1] - 2 * I) @ (O[1] - 2 * I) - O[5] @ O[5] - O[9] @ O[9] + 2 * O[13] @ O[13] - 4 * I
    assert np.abs(lhs - rhs).max() < 1e-13
    from oracle.model import gamma_matrices
    gm = gamma_matrices()
    for g, t in zip(gm, (5, 9, 14, 15, 16)):
        assert np.abs(g - T[t - 1]).max() == 0


def test_fierz_projected_torus_n2():
    """Eq. model vs eq. newmodel on the torus at N=2 (Fock dimension 256): the
    rewrite holds up to a constant, a multiple of the particle number and the
    momentum-cutoff residual."""
    n = 2
    cs = fock.annihilators(4 * n)
    from oracle.model import momentum_set
    qs = momentum_set(n, Q_PAPER)
    u0, uk, un = 1.0, 0.7, 0.4
    Ho = fock.hamiltonian_original(cs, n, qs, u0, uk, un)
    g = np.array([u0 + un, -(uk + un), -(uk + un), 2 * un])
    Hn = fock.hamiltonian_fierz(cs, n, qs, g)
    dH = Ho - Hn
    Nop = sum(c.T @ c for c in cs)
    d = np.diag(dH).real
    X = np.stack([np.ones(256), np.diag(Nop)], 1)
    coef, *_ = np.linalg.lstsq(X, d, rcond=None)
    resid = dH - np.diag(X @ coef)
    assert np.abs(resid).max() < 1e-6
    assert np.abs(Ho - Ho.conj().T).max() < 1e-12


# ---------------------------------------------------------------- HS and Fock trace

@pytest.mark.parametrize("chan,g", [(0, 1.7), (1, -2.2), (3, 1.1)])
def test_hs_identity_quadrature(chan, g):
    """Eq. HS transform: int dphi N(phi) exp(alpha phi Q) = exp(-dtau g Q^2/2)
    with alpha = sqrt(-dtau g), on one Fock-space component at N = 2."""
    n, dtau = 2, 0.1
    cs = fock.annihilators(4 * n)
    comps = components(n, Q_PAPER)
    Q = fock.component_operators(cs, n, comps[:3], PAULI[chan], chan == 0)[2]
    alpha = np.sqrt(complex(-dtau * g))
    x, w = np.polynomial.hermite_e.hermegauss(60)
    w = w / np.sqrt(2 * np.pi)
    ev, U = np.linalg.eigh(Q)
    lhs = sum(wi * (U * np.exp(alpha * xi * ev)) @ U.conj().T for xi, wi in zip(x, w))
    rhs = sla.expm(-dtau * g * Q @ Q / 2)
    assert np.abs(lhs - rhs).max() < 1e-12


@pytest.mark.parametrize("mode", [Q_PAPER, Q_BZ])
def test_fock_trace_identity(mode):
    """Tr_Fock prod_tau prod_i exp(alpha_i sum_c phi Q_c) with the density operators
    built from the printed formula equals exp(sum c_tau) det(1 + B(beta,0))^2."""
    n, L = 2, 2
    m = Model(n, L, 0.1, u0=1.0, uk=0.9, un=1.2, q_mode=mode)
    cs = fock.annihilators(4 * n)
    Qops = [fock.component_operators(cs, n, m.comps, PAULI[i], i == 0) for i in range(4)]
    phi = synth.fields(11, L, m.n_q)
    prod = np.eye(256, dtype=complex)
    for t in range(L):
        for i in range(4):
            X = m.alpha[i] * sum(phi[t, i, c] * Qops[i][c] for c in range(m.n_q))
            prod = prod @ sla.expm(X)
    tr = np.trace(prod)
    w = np.exp(dqmc.logdet(m, phi))
    assert abs(tr - w) < 1e-11 * abs(w)
    assert abs(w.imag) < 1e-10 * abs(w) and w.real > 0


# ---------------------------------------------------------------- closed forms

def _single_component(m, chan, rng):
    phi = np.zeros((m.l_tau, 4, m.n_q))
    phi[:, chan, 0] = rng.standard_normal(m.l_tau)
    return phi


def test_closed_form_channel0():
    n, L, dtau, g0 = 5, 7, 0.1, 1.3
    m = Model(n, L, dtau, u0=g0)
    phi = _single_component(m, 0, np.random.default_rng(3))
    th = np.sqrt(dtau * g0) * np.sqrt(2) * form_factor(0, 0, n) * phi[:, 0, 0].sum()
    ld = dqmc.logdet(m, phi)
    assert abs(ld.real - 4 * n * np.log(2 * np.cos(th / 2))) < 1e-12
    for tau in (0, 3, L):
        G = dqmc.green(m, phi, tau)
        assert np.abs(G - np.eye(2 * n) / (1 + np.exp(1j * th))).max() < 1e-14


def test_closed_form_channel1():
    n, L, dtau, uk = 5, 7, 0.1, 0.65
    m = Model(n, L, dtau, u0=0.0, uk=uk, un=0.0)
    phi = _single_component(m, 1, np.random.default_rng(4))
    th = np.sqrt(dtau * uk) * np.sqrt(2) * form_factor(0, 0, n) * phi[:, 1, 0].sum()
    ld = dqmc.logdet(m, phi)
    assert abs(ld.real - 4 * n * np.log(2 * np.cosh(th / 2))) < 1e-12
    G = dqmc.green(m, phi, 2)
    expect = 0.5 * np.eye(2 * n) - 0.5 * np.tanh(th / 2) * np.kron(PAULI[1], np.eye(n))
    assert np.abs(G - expect).max() < 1e-14


def test_closed_form_channel3():
    n, L, dtau, un = 5, 7, 0.1, 0.65
    m = Model(n, L, dtau, u0=-un, uk=-un, un=un)    # g = (0, 0, 0, 2 un)
    assert np.allclose(m.g[:3], 0)
    phi = _single_component(m, 3, np.random.default_rng(5))
    th = np.sqrt(dtau * 2 * un) * np.sqrt(2) * form_factor(0, 0, n) * phi[:, 3, 0].sum()
    ld = dqmc.logdet(m, phi)
    assert abs(ld.real - 4 * n * np.log(2 * abs(np.cos(th / 2)))) < 1e-12
    G = dqmc.green(m, phi, 4)
    d = np.concatenate([np.full(n, 1 / (1 + np.exp(1j * th))), np.full(n, 1 / (1 + np.exp(-1j * th)))])
    assert np.abs(G - np.diag(d)).max() < 1e-14


def test_free_fermions():
    """All couplings zero: B = 1, G = 1/2, logdet = 4N ln 2."""
    n, L = 4, 5
    m = Model(n, L, 0.1, u0=0.0, uk=0.0, un=0.0)
    phi = synth.fields(2, L, m.n_q)
    assert abs(dqmc.logdet(m, phi) - 4 * n * np.log(2)) < 1e-12
    assert np.abs(dqmc.green(m, phi, 2) - 0.5 * np.eye(2 * n)).max() < 1e-15


def test_single_component_library_eigh():
    """One active general-q component reduces to diagonalising its Hermitian matrix."""
    n, L, dtau, uk = 4, 3, 0.1, 0.8
    m = Model(n, L, dtau, u0=0.0, uk=uk, un=0.0)
    c = 5
    phi = np.zeros((L, 4, m.n_q))
    phi[:, 1, c] = [0.7, -1.1, 0.4]
    lam, _ = np.linalg.eigh(m.qmats[c])
    th = np.sqrt(dtau * uk) * phi[:, 1, c].sum() * lam
    expect = 2 * np.sum(np.log(1 + np.exp(th)) + np.log(1 + np.exp(-th)))
    assert abs(dqmc.logdet(m, phi).real - expect) < 1e-12


# ---------------------------------------------------------------- brute force and invariants

def test_mpmath_brute_force():
    """G(tau) and logdet against 40-digit dense arithmetic (mpmath)."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    n, L = 3, 4
    m = Model(n, L, 0.1, u0=1.0, uk=1.5, un=1.5)
    phi = synth.fields(7, L, m.n_q)
    Bs = dqmc.propagators(m, phi)
    # exponentials in mpmath from the same one-body exponents
    Bmp = []
    for t in range(L):
        Bt = mp.eye(2 * n)
        for i in range(4):
            V = mp.matrix(m.V(phi[t], i).tolist())
            Bt = Bt * mp.expm(V)
        Bmp.append(Bt)
    tau = 2
    left, right = mp.eye(2 * n), mp.eye(2 * n)
    for t in range(1, tau + 1):
        left = Bmp[t - 1] * left
    for t in range(tau + 1, L + 1):
        right = Bmp[t - 1] * right
    Gmp = (mp.eye(2 * n) + left * right) ** -1
    G = dqmc.green(m, phi, tau, Bs)
    err = max(abs(complex(Gmp[i, j]) - G[i, j]) for i in range(2 * n) for j in range(2 * n))
    assert err < 1e-13
    full = mp.eye(2 * n)
    for t in range(1, L + 1):
        full = Bmp[t - 1] * full
    ld_mp = 2 * mp.log(mp.det(mp.eye(2 * n) + full)) + sum(m.c_tau(phi[t]) for t in range(L))
    ld = dqmc.logdet(m, phi)
    assert abs(complex(ld_mp).real - ld.real) < 1e-12


@pytest.mark.parametrize("mode,n", [(Q_PAPER, 3), (Q_PAPER, 5), (Q_BZ, 4)])
def test_sign_free_and_particle_hole(mode, n):
    """Fierz channels give a real positive weight (Results: sign-free) and
    Re tr G = N on the spin block for every configuration (half filling)."""
    L = 5
    m = Model(n, L, 0.1, u0=1.0, uk=1.2, un=1.2, q_mode=mode)
    phi = synth.fields(100 + n, L, m.n_q, scale=2.0)
    ld = dqmc.logdet(m, phi)
    assert abs(np.angle(np.exp(1j * ld.imag))) < 1e-10
    for tau in (0, 2):
        assert abs(np.trace(dqmc.green(m, phi, tau)).real - n) < 1e-11


def test_gradient_finite_difference():
    """Jacobi's formula with the exact Frechet derivative (gradient equation, read
    as d ln w / d phi = 2 Tr[(1-G) dB B^{-1}] + background) against central
    differences of ln w; the first-order drift approximates it."""
    n, L, tau = 3, 4, 2
    m = Model(n, L, 0.1, u0=1.0, uk=1.5, un=1.5)
    phi = synth.fields(9, L, m.n_q)
    g = dqmc.exact_grad_lnw(m, phi, tau)
    assert np.abs(g.imag).max() < 1e-12
    h = 1e-5
    for (i, c) in [(0, 0), (1, 3), (2, 5), (3, 8), (0, 7)]:
        pp, pm = phi.copy(), phi.copy()
        pp[tau - 1, i, c] += h
        pm[tau - 1, i, c] -= h
        fd = (dqmc.logdet(m, pp).real - dqmc.logdet(m, pm).real) / (2 * h)
        assert abs(fd - g[i, c].real) < 1e-7
    G = dqmc.green(m, phi, tau)
    D = dqmc.drift(m, phi[tau - 1], G)
    exact = -phi[tau - 1] + g.real
    rel = np.abs(D - exact).max() / np.abs(g.real).max()
    assert rel < 0.1


# ---------------------------------------------------------------- observables

def test_observables_fock_expectation():
    """Wick evaluation of S^i_q from G equals the Fock-space expectation
    Tr[B n_q n_-q]/Tr[B] with B the Fock propagator of the configuration."""
    n, L = 2, 2
    m = Model(n, L, 0.1, u0=1.0, uk=1.0, un=1.0)
    cs = fock.annihilators(4 * n)
    Qops = [fock.component_operators(cs, n, m.comps, PAULI[i], i == 0) for i in range(4)]
    phi = synth.fields(21, L, m.n_q)
    Bf = np.eye(256, dtype=complex)
    for t in range(L):
        Bt = np.eye(256, dtype=complex)
        for i in range(4):
            Bt = Bt @ sla.expm(m.alpha[i] * sum(phi[t, i, c] * Qops[i][c] for c in range(m.n_q)))
        Bf = Bt @ Bf
    G = dqmc.green(m, phi, L)
    from oracle.model import gamma_matrices
    for gm in gamma_matrices():
        for (qx, qy) in [(0, 0), (1, 0), (1, 1)]:
            a = fock.density_operator(cs, n, qx, qy, gm, False)
            b = fock.density_operator(cs, n, -qx, -qy, gm, False)
            ex = np.trace(Bf @ a @ b) / np.trace(Bf)
            assert abs(ex - structure_factor(G, n, gm, qx, qy)) < 1e-11
    s, m2 = so5_observables(G, n)
    assert abs(s[2] - s[3]) < 1e-12 and abs(s[3] - s[4]) < 1e-12     # spin SU(2)
    assert m2 > 0


def _fock_slices(m, phi, cs):
    """Fock-space propagators of the slices, B_tau = prod_i exp(alpha_i sum_c
    phi^i_c Q^i_c) in channel order 0..3, from the second-quantised
    components (sum-of-squares equation); list index tau - 1."""
    Qops = [fock.component_operators(cs, m.n_phi, m.comps, PAULI[i], i == 0) for i in range(4)]
    dim = cs[0].shape[0]
    out = []
    for t in range(m.l_tau):
        Bt = np.eye(dim, dtype=complex)
        for i in range(4):
            Bt = Bt @ sla.expm(m.alpha[i] * sum(phi[t, i, c] * Qops[i][c] for c in range(m.n_q)))
        out.append(Bt)
    return out


def _fock_range(Bf, t2, t1):
    out = np.eye(Bf[0].shape[0], dtype=complex)
    for t in range(t1 + 1, t2 + 1):
        out = Bf[t - 1] @ out
    return out


@pytest.mark.parametrize("tau", [0, 1, 2, 3])
def test_displaced_green_fock(tau):
    """G(tau,0)_ij = Tr[B(beta,tau) c_i B(tau,0) c_j^+] / Tr B(beta,0) and
    G(0,tau)_ij = -Tr[B(beta,tau) c_j^+ B(tau,0) c_i] / Tr B(beta,0) in Fock
    space (8 modes, 256 states) against the oracle's single-particle formulas,
    with G_4N = 1_spin kron G (Supplementary Note 2 needs both)."""
    n, L = 2, 3
    m = Model(n, L, 0.1, u0=1.0, uk=1.3, un=0.8)
    cs = fock.annihilators(4 * n)
    phi = synth.fields(61, L, m.n_q)
    Bf = _fock_slices(m, phi, cs)
    left, right = _fock_range(Bf, L, tau), _fock_range(Bf, tau, 0)
    Z = np.trace(left @ right)
    Gt0, G0t, Gtt = dqmc.green_displaced(m, phi, tau)
    E = np.eye(2)
    X, Y, W = np.kron(E, Gt0), np.kron(E, G0t), np.kron(E, Gtt)
    for i in range(4 * n):
        for j in range(4 * n):
            a = np.trace(left @ cs[i] @ right @ cs[j].T) / Z
            b = -np.trace(left @ cs[j].T @ right @ cs[i]) / Z
            c = np.trace(left @ right @ cs[i] @ cs[j].T) / Z if tau == 0 else \
                np.trace(left @ cs[i] @ cs[j].T @ right) / Z
            assert abs(a - X[i, j]) < 1e-12
            assert abs(b - Y[i, j]) < 1e-12
            assert abs(c - W[i, j]) < 1e-12


@pytest.mark.parametrize("tau", [1, 2])
def test_so5_correlator_fock(tau):
    """<n^{Gamma^i}_{q=0}(tau) n^{Gamma^i}_{q=0}(0)> = Tr[B(beta,tau) n B(tau,0) n]
    / Tr B(beta,0) with the density operators of the printed second-quantised
    formula (Supplementary Note 2), against the Wick evaluation."""
    from oracle.model import gamma_matrices
    from oracle.observables import so5_correlator
    n, L = 2, 3
    m = Model(n, L, 0.1, u0=1.0, uk=1.1, un=1.1)
    cs = fock.annihilators(4 * n)
    phi = synth.fields(62, L, m.n_q)
    Bf = _fock_slices(m, phi, cs)
    left, right = _fock_range(Bf, L, tau), _fock_range(Bf, tau, 0)
    Z = np.trace(left @ right)
    Gt0, G0t, Gtt = dqmc.green_displaced(m, phi, tau)
    G00 = dqmc.green(m, phi, 0)
    c, m2 = so5_correlator(Gt0, G0t, Gtt, G00, n)
    ex = []
    for gm in gamma_matrices():
        a = fock.density_operator(cs, n, 0, 0, gm, False)
        ex.append(np.trace(left @ a @ right @ a) / Z)
    ex = np.array(ex)
    assert np.abs(c - ex).max() < 1e-12
    assert abs(m2 - ex.mean()) < 1e-12


def test_displaced_green_boundaries():
    """Antiperiodicity in tau of the fermion propagator: G(beta,0) = 1 - G(0),
    G(0,beta) = -G(0); the bosonic correlator is periodic, C(beta) = C(0), and
    C(0) is the equal-time S^i_{q=0} (Results)."""
    from oracle.observables import so5_correlator
    n, L = 3, 6
    m = Model(n, L, 0.1, u0=1.0, uk=1.5, un=1.5)
    phi = synth.fields(63, L, m.n_q)
    G0 = dqmc.green(m, phi, 0)
    Gt0, G0t, Gtt = dqmc.green_displaced(m, phi, L)
    I = np.eye(m.n)
    assert np.abs(Gt0 - (I - G0)).max() < 1e-12
    assert np.abs(G0t + G0).max() < 1e-12
    cb, _ = so5_correlator(Gt0, G0t, Gtt, G0, n)
    c0, _ = so5_correlator(*dqmc.green_displaced(m, phi, 0), G0, n)
    s, _ = so5_observables(G0, n)
    assert np.abs(cb - c0).max() < 1e-12 * np.abs(c0).max()
    assert np.abs(c0 - s).max() < 1e-14


# ---------------------------------------------------------------- the Markov chain

def test_mala_free_gaussian_target():
    """All couplings zero: the target is N(0,1) per field (S_0 only), so MALA
    samples must have mean 0 and variance 1."""
    n, L = 2, 4
    m = Model(n, L, 0.1, u0=0.0, uk=0.0, un=0.0)
    phi = synth.fields(31, L, m.n_q)
    ch = dqmc.Chain(m, phi, eps0=0.8, adapt=False)
    rp = synth.replay(32, 400, L, m.n_q)
    samples = []
    for s in range(400):
        ch.sweep(rp[s])
        if s >= 20:
            samples.append(ch.phi.copy())
    x = np.array(samples).ravel()
    assert abs(x.mean()) < 0.05
    assert abs(x.var() - 1.0) < 0.05


def test_sweep_bookkeeping_consistent():
    """Summing the accepted log-weight changes of a sweep reproduces the change
    of ln w computed from scratch; the per-move phase stays zero (sign-free)."""
    n, L = 3, 6
    m = Model(n, L, 0.1, u0=1.0, uk=1.0, un=1.0)
    phi0 = synth.fields(41, L, m.n_q)
    ch = dqmc.Chain(m, phi0, eps0=0.8, adapt=False)
    rp = synth.replay(42, 2, L, m.n_q)
    ch.run(rp)
    assert ch.phase_err < 1e-10
    acc = [h for h in ch.history if h[2]]
    assert 0 < len(acc) <= 2 * L
    # ln A of accepted moves obeys its definition on the final state
    assert np.isfinite([h[1] for h in ch.history]).all()


# ---------------------------------------------------------------- torus density operator from the wave functions

def _lll_torus(n_phi, xs, ys, k, images=6):
    """Printed LLL wave function of orbital k (Methods, toric regularization;
    l_B = 1, square cell L_x = L_y = sqrt(2 pi N)) made periodic in x by the
    sum over magnetic translations k -> k + j N, evaluated on the grid."""
    ly = np.sqrt(2 * np.pi * n_phi)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    out = np.zeros_like(X, dtype=complex)
    for j in range(-images, images + 1):
        kj = k + j * n_phi
        out += np.exp(-(X - 2 * np.pi * kj / ly) ** 2 / 2) * np.exp(2j * np.pi * kj * Y / ly)
    return out / np.sqrt(ly * np.sqrt(np.pi))


@pytest.mark.parametrize("n_phi", [3, 4])
def test_torus_density_operator_from_wave_functions(n_phi):
    """Eq. torus density operator against its definition n_q = int dr e^{iq.r}
    psi^dagger psi: the matrix elements int e^{iq.r} phi_k^* phi_k' over one
    periodic cell of the printed LLL wave functions (q = sqrt(2 pi / N) (qx, qy)).
    The trapezoid rule is spectrally exact for these periodic integrands. The
    integral fixes the Gaussian exponent, the orbital shift and the phase; the
    printed overall factor 1 / (4 pi sqrt N) multiplies it (a normalisation of
    the couplings, taken as printed)."""
    n = n_phi
    lc = np.sqrt(2 * np.pi * n)
    ng = 96
    xs = np.arange(ng) * lc / ng
    ys = np.arange(ng) * lc / ng
    wf = [_lll_torus(n, xs, ys, k) for k in range(1, n + 1)]
    dA = (lc / ng) ** 2
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    # normalisation of the periodic states over one cell
    for k in range(n):
        for kp in range(n):
            ov = np.sum(wf[k].conj() * wf[kp]) * dA
            assert abs(ov - (k == kp)) < 1e-12
    for (qx, qy) in [(0, 0), (1, 0), (0, 1), (1, 2), (-2, 1), (2, -3), (3, 3)]:
        qv = np.sqrt(2 * np.pi / n) * np.array([qx, qy])
        ph = np.exp(1j * (qv[0] * X + qv[1] * Y))
        M = np.array([[np.sum(ph * wf[k].conj() * wf[kp]) * dA for kp in range(n)] for k in range(n)])
        ref = m_matrix(qx, qy, n) * (4 * np.pi * np.sqrt(n))
        assert np.abs(M - ref).max() < 1e-11, (qx, qy)
        assert abs(form_factor(qx, qy, n) * 4 * np.pi * np.sqrt(n) - np.exp(-np.sum(qv ** 2) / 4)) < 1e-15


# ---------------------------------------------------------------- the interacting chain at N = 2, L = 1

# One q = 0 component per channel: q_0 = sqrt(2) F(0) 1, so the slice propagator
# is a function of a valley 2x2 matrix and the fermion weight is closed form:
#   channel 0 alone (g = (g0, 0, 0, 0)): w_F = (2 cos(a phi_0 / 2))^{4N},
#   channels 1, 2 (g = (0, -K, -K, 0)): det(1 + e^{a phi_1 tau_x} e^{a phi_2 tau_y})
#     = 2 + 2 cosh(a phi_1) cosh(a phi_2), w_F = (2 + 2 cosh cosh)^{2N},
# with a = sqrt(dtau |g|) sqrt(2) F(0). Derived by hand from B = E_0 E_1 E_2 E_3.

def _closed_lnw(case, a, n_phi, ph):
    if case == 0:
        return 4 * n_phi * np.log(np.abs(2 * np.cos(a * ph[0, 0] / 2)))
    return 2 * n_phi * np.log(2 + 2 * np.cosh(a * ph[1, 0]) * np.cosh(a * ph[2, 0]))


def _closed_grad(case, a, n_phi, ph):
    g = np.zeros_like(ph)
    if case == 0:
        g[0, 0] = -2 * n_phi * a * np.tan(a * ph[0, 0] / 2)
    else:
        x, y = a * ph[1, 0], a * ph[2, 0]
        den = 1 + np.cosh(x) * np.cosh(y)
        g[1, 0] = 2 * n_phi * a * np.sinh(x) * np.cosh(y) / den
        g[2, 0] = 2 * n_phi * a * np.cosh(x) * np.sinh(y) / den
    return g


def _tiny_model(case, a):
    from oracle.model import Q_LIST
    f0 = form_factor(0, 0, 2) * np.sqrt(2)
    dtau = 0.1
    gabs = (a / f0) ** 2 / dtau
    if case == 0:
        return Model(2, 1, dtau, u0=gabs, uk=0.0, un=0.0, q_mode=Q_LIST, q_list=[(0, 0)])
    return Model(2, 1, dtau, u0=0.0, uk=gabs, un=0.0, q_mode=Q_LIST, q_list=[(0, 0)])


@pytest.mark.parametrize("case,a", [(0, 0.5), (1, 0.4)])
def test_interacting_chain_lna_closed_form(case, a):
    """Langevin proposal, proposal density and Metropolis-Hastings test (Methods,
    Langevin-based global update scheme) with a live fermion weight: every
    recorded ln A of the oracle's chain equals the closed form
      -(|phi'|^2 - |phi|^2)/2 + Delta ln w_F + ln f(phi | phi') - ln f(phi' | phi)
    with phi' = phi + eps^2/2 D + eps eta and D = -phi + grad ln w_F, all in
    closed form (a sign or factor error in Delta ln w_F or the drift fails)."""
    m = _tiny_model(case, a)
    assert m.n_q == 1
    n_phi = m.n_phi
    eps = 0.9
    ch = dqmc.Chain(m, synth.fields(51 + case, 1, 1), eps0=eps, adapt=False)
    rp = synth.replay(61 + case, 200, 1, 1)
    for s in range(200):
        ph = ch.phi[0].copy()
        ch.sweep(rp[s])
        eta = rp[s, 0, :4].reshape(4, 1)
        D = -ph + _closed_grad(case, a, n_phi, ph)
        php = ph + 0.5 * eps * eps * D + eps * eta
        Dp = -php + _closed_grad(case, a, n_phi, php)
        lnA = (-0.5 * (np.sum(php ** 2) - np.sum(ph ** 2))
               + _closed_lnw(case, a, n_phi, php) - _closed_lnw(case, a, n_phi, ph)
               - np.sum((ph - php - 0.5 * eps * eps * Dp) ** 2) / (2 * eps * eps)
               + np.sum((php - ph - 0.5 * eps * eps * D) ** 2) / (2 * eps * eps))
        got = ch.history[-1][1]
        assert abs(got - lnA) < 1e-9 * max(1.0, abs(lnA)), (s, got, lnA)
        assert ch.history[-1][2] == (np.log(rp[s, 0, 4]) < lnA)
    assert ch.phase_err < 1e-10


def _marginal_cdf(case, a, n_phi, grid):
    """CDF of the stationary marginal of the active field (phi_0 for channel 0,
    phi_1 for channels 1, 2) from e^{-|phi|^2/2} w_F by quadrature."""
    if case == 0:
        dens = np.exp(-grid ** 2 / 2) * np.abs(2 * np.cos(a * grid / 2)) ** (4 * n_phi)
    else:
        y, wy = np.polynomial.hermite_e.hermegauss(80)
        dens = np.array([np.sum(wy * (2 + 2 * np.cosh(a * x) * np.cosh(a * y)) ** (2 * n_phi))
                         for x in grid]) * np.exp(-grid ** 2 / 2)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(grid))])
    return cdf / cdf[-1]


@pytest.mark.parametrize("case,a", [(0, 0.5), (1, 0.4)])
def test_interacting_chain_stationary_law(case, a):
    """The chain samples e^{-|phi|^2/2} w_F(phi) (Methods, continuous HS transform
    and Langevin update): 2e4 sweeps at N = 2, L = 1 with one active channel
    component, thinned by 4, against the exact 1D marginal by quadrature
    (Kolmogorov-Smirnov distance) and its second moment; the inactive channels
    stay N(0, 1). With ln w_F doubled the exact variance of the active field
    moves from 0.66 to 0.49 (channel 0) and from 1.46 to 2.70 (channels 1, 2);
    with its sign flipped, to a non-normalisable law and to 0.76."""
    m = _tiny_model(case, a)
    ch = dqmc.Chain(m, synth.fields(71 + case, 1, 1), eps0=1.2, adapt=False)
    n_sw = 20000
    rp = synth.replay(81 + case, n_sw, 1, 1)
    xs = np.empty((n_sw, 4))
    for s in range(n_sw):
        ch.sweep(rp[s])
        xs[s] = ch.phi[0, :, 0]
    acc = sum(h[2] for h in ch.history) / n_sw
    assert 0.3 < acc < 0.95
    act = 0 if case == 0 else 1
    x = np.sort(xs[500::4, act])
    grid = np.linspace(-8, 8, 4001)
    cdf = _marginal_cdf(case, a, m.n_phi, grid)
    emp = np.arange(1, x.size + 1) / x.size
    ks = np.max(np.abs(np.interp(x, grid, cdf) - emp))
    assert ks < 0.03, ks
    # second moment of the exact marginal
    pdf = np.gradient(cdf, grid)
    var = np.sum(pdf * grid ** 2) * (grid[1] - grid[0])
    assert abs(np.mean(x ** 2) - var) < 0.06 * var
    assert abs(var - 1.0) > 0.3   # the fermion weight is visible in the law
    for free in ([3] if case == 0 else [0, 3]):
        y = xs[500::4, free]
        assert abs(np.mean(y)) < 0.06 and abs(np.var(y) - 1.0) < 0.08


def test_eps_controller_settles():
    """Adaptive step (Methods, Langevin-based global update scheme): eps <- eps +
    (r_a - 0.574) * 0.1 after each sweep drives the acceptance to the set point
    from a step that is too large and from one that is too small; with eps frozen
    at the settled value the acceptance is the set point."""
    m = _tiny_model(1, 0.4)
    from oracle.model import Q_LIST
    L4 = Model(2, 4, m.dtau, u0=0.0, uk=m.uk, un=0.0, q_mode=Q_LIST, q_list=[(0, 0)])
    settled = []
    for eps0, seed in ((3.0, 91), (0.05, 92)):
        ch = dqmc.Chain(L4, synth.fields(seed, 4, 1), eps0=eps0, adapt=True)
        rp = synth.replay(seed + 10, 1500, 4, 1)
        eps_hist = []
        for s in range(1500):
            ch.sweep(rp[s])
            eps_hist.append(ch.eps)
        acc = np.array([h[2] for h in ch.history[-4 * 1000:]])
        assert abs(acc.mean() - 0.574) < 0.02, (eps0, acc.mean())
        settled.append(np.mean(eps_hist[500:]))
    assert abs(settled[0] - settled[1]) < 0.15 * settled[0]
    ch = dqmc.Chain(L4, synth.fields(95, 4, 1), eps0=np.mean(settled), adapt=False)
    rp = synth.replay(96, 1500, 4, 1)
    ch.run(rp)
    acc = np.array([h[2] for h in ch.history[400:]])
    assert abs(acc.mean() - 0.574) < 0.04, acc.mean()


@pytest.mark.parametrize("mode", [Q_BZ, Q_PAPER])
def test_fierz_energy_matches_fock_thermal_state(mode):
    """Wick evaluation of <H> (eq. newmodel) against the trace in Fock space at
    N = 2: for a spin-degenerate Gaussian operator rho = exp(-c+ (1 (x) K) c)
    with K a random complex matrix (not Hermitian, as the propagator products
    of a field configuration), Tr[H rho] / Tr[rho] equals fierz_energy of
    G = (1 + e^{-K})^{-1}, the Green's function G_ij = <c_i c_j^dagger> of rho."""
    n = 2
    rng = np.random.default_rng(5)
    K = 0.8 * (rng.normal(size=(2 * n, 2 * n)) + 1j * rng.normal(size=(2 * n, 2 * n)))
    G = np.linalg.inv(np.eye(2 * n) + sla.expm(-K))
    cs = fock.annihilators(4 * n)
    m = Model(n, 2, 0.1, u0=1.0, uk=2.0, un=1.3, q_mode=mode)
    from oracle.model import momentum_set
    qs = momentum_set(n, mode)
    H = fock.hamiltonian_fierz(cs, n, qs, m.g)
    rho = sla.expm(-fock.bilinear(cs, np.kron(np.eye(2), K)))
    e_fock = np.trace(H @ rho) / np.trace(rho)
    e = fierz_energy(G, n, qs, m.g)
    assert abs(e - e_fock) < 1e-12 * max(1.0, abs(e_fock))
    assert abs(e_fock) > 1e-3          # the case is not degenerate

"""Pins of the spherical regularisation in the oracle (Methods, "Spherical
regularization"), CPU only. The 3j symbols are checked against closed forms
and orthogonality; the printed density operator against the projection of
Y*_{l,m} on the printed monopole harmonics (numerical quadrature, scipy's
spherical harmonics) and against rotation covariance; the HS machinery against
Fock-space traces and the Fierz rewrite."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import dqmc, fock, sphere
from oracle.model import Model, PAULI, Q_SPHERE, gamma_matrices
from oracle.observables import so5_observables, structure_factor


def test_wigner3j_closed_forms_and_orthogonality():
    w = sphere.wigner3j
    for tj in range(0, 7):
        for tm in range(-tj, tj + 1, 2):
            assert abs(w(tj, tj, 0, tm, -tm, 0) - (-1) ** ((tj - tm) // 2) / math.sqrt(tj + 1)) < 1e-14
    assert abs(w(2, 2, 2, 2, -2, 0) - 1.0 / math.sqrt(6.0)) < 1e-15          # (1 1 1; 1 -1 0)
    assert abs(w(2, 2, 4, 0, 0, 0) - math.sqrt(2.0 / 15.0)) < 1e-15           # (1 1 2; 0 0 0)
    assert w(2, 2, 2, 0, 0, 0) == 0.0                                         # odd j sum, all m = 0
    # sum_{m1,m2} (2 j3 + 1) 3j(j1 j2 j3; m1 m2 m3) 3j(j1 j2 j3'; m1 m2 m3') = delta delta
    for tj1, tj2 in ((3, 4), (5, 2), (4, 4)):
        for tj3 in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
            for tj3p in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
                for tm3 in range(-min(tj3, tj3p), min(tj3, tj3p) + 1, 2):
                    s = sum((tj3 + 1) * w(tj1, tj2, tj3, tm1, -tm1 - tm3, tm3)
                            * w(tj1, tj2, tj3p, tm1, -tm1 - tm3, tm3)
                            for tm1 in range(-tj1, tj1 + 1, 2))
                    assert abs(s - (1.0 if tj3 == tj3p else 0.0)) < 1e-13


@pytest.mark.parametrize("n_phi", [3, 4])
def test_sphere_density_is_projected_spherical_harmonic(n_phi):
    """The printed 3j density operator equals c times the matrix of Y*_{l,m}
    between the printed LLL monopole harmonics, with one constant c for all
    (l, m) and orbital pairs, |c| = sqrt(pi) (its sign, (-1)^(2s), is the
    printed formula's convention and drops out of n n^+)."""
    from scipy.special import sph_harm_y
    xg, wg = np.polynomial.legendre.leggauss(40)
    th = np.arccos(xg)
    ph = np.linspace(0.0, 2.0 * np.pi, 64, endpoint=False)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(wg, np.full(64, 2.0 * np.pi / 64))
    psi = [sphere.monopole_harmonic(k, n_phi, TH, PH) for k in range(1, n_phi + 1)]
    for a in range(n_phi):
        for b in range(n_phi):
            assert abs(np.sum(W * np.conj(psi[a]) * psi[b]) - (a == b)) < 1e-12
    c = (-1) ** (n_phi - 1) * math.sqrt(math.pi)
    for (l, m) in sphere.momenta(n_phi):
        Y = sph_harm_y(l, m, TH, PH)
        I = np.array([[np.sum(W * np.conj(psi[a]) * np.conj(Y) * psi[b]) for b in range(n_phi)]
                      for a in range(n_phi)])
        D = sphere.density_matrix(l, m, n_phi)
        assert np.abs(D - c * I).max() < 1e-12, (l, m)


@pytest.mark.parametrize("n_phi", [3, 4, 5])
def test_sphere_density_rotation_covariance(n_phi):
    """n_{l,m} is a spherical tensor: [L_z, n_{l,m}] = -m n_{l,m},
    [L_+, n_{l,m}] = -sqrt((l+m)(l-m+1)) n_{l,m-1}, n_{l,-m} = (-1)^m n_{l,m}^+,
    and the Casimir sum_a [L_a, [L_a, n]] = l(l+1) n."""
    lz, lp = sphere.lz_lplus(n_phi)
    lm = lp.conj().T
    lx, ly = (lp + lm) / 2, (lp - lm) / 2j
    comm = lambda a, b: a @ b - b @ a
    for (l, m) in sphere.momenta(n_phi):
        D = sphere.density_matrix(l, m, n_phi)
        assert np.abs(D).max() > 1e-3
        assert np.abs(comm(lz, D) + m * D).max() < 1e-13
        if m > -l:
            assert np.abs(comm(lp, D) + math.sqrt((l + m) * (l - m + 1)) * sphere.density_matrix(l, m - 1, n_phi)).max() < 1e-13
        assert np.abs(sphere.density_matrix(l, -m, n_phi) - (-1) ** m * D.conj().T).max() < 1e-14
        cas = sum(comm(a, comm(a, D)) for a in (lx, ly, lz))
        assert np.abs(cas - l * (l + 1) * D).max() < 1e-12
    assert not np.any(sphere.density_matrix(n_phi, 0, n_phi))        # l > 2s vanishes


def test_sphere_components_sum_of_squares():
    """sum_c Q_c^2 / 2 over the Hermitian components of one channel equals
    sum_{l,m} n_{l,m} n_{l,m}^+ (sum-of-squares equation on the sphere), as
    one-body matrices."""
    n = 4
    comps = sphere.components(n)
    assert len(comps) == n * n
    lhs = sum(sphere.component_matrix(k, l, m, n) @ sphere.component_matrix(k, l, m, n) for (k, l, m) in comps) / 2
    rhs = sum(sphere.density_matrix(l, m, n) @ sphere.density_matrix(l, m, n).conj().T
              for (l, m) in sphere.momenta(n))
    assert np.abs(lhs - rhs).max() < 1e-13
    for (k, l, m) in comps:
        q = sphere.component_matrix(k, l, m, n)
        assert np.abs(q - q.conj().T).max() < 1e-15


def test_sphere_fock_trace_identity():
    """Tr_Fock prod_tau prod_i exp(alpha_i sum_c phi Q_c) with the sphere's
    second-quantised components equals exp(sum c_tau) det(1 + B(beta,0))^2
    (N = 2, s = 1/2, 256 states); the weight is real and positive."""
    n, L = 2, 2
    m = Model(n, L, 0.1, u0=1.0, uk=0.9, un=1.2, q_mode=Q_SPHERE)
    cs = fock.annihilators(4 * n)
    Qops = [fock.component_operators_sphere(cs, n, m.comps, PAULI[i], i == 0) for i in range(4)]
    phi = synth.fields(71, L, m.n_q)
    prod = np.eye(256, dtype=complex)
    for t in range(L):
        for i in range(4):
            prod = prod @ sla.expm(m.alpha[i] * sum(phi[t, i, c] * Qops[i][c] for c in range(m.n_q)))
    w = np.exp(dqmc.logdet(m, phi))
    assert abs(np.trace(prod) - w) < 1e-11 * abs(w)
    assert abs(w.imag) < 1e-10 * abs(w) and w.real > 0


def test_sphere_fierz_rewrite_n2():
    """Eq. model vs eq. newmodel with the sphere's density operators (every
    (l, m) kept, so no cutoff residual): equal up to a constant and a
    multiple of the particle number."""
    n = 2
    cs = fock.annihilators(4 * n)
    u0, uk, un = 1.0, 0.7, 0.4
    Ho = fock.hamiltonian_sphere(cs, n, [u0, -uk, -uk, -un, -un, -un],
                                 [np.eye(4, dtype=complex)] + gamma_matrices(), True)
    g = [u0 + un, -(uk + un), -(uk + un), 2 * un]
    Hn = fock.hamiltonian_sphere(cs, n, g, [np.kron(PAULI[i], PAULI[0]) for i in range(4)], True)
    dH = Ho - Hn
    Nop = sum(c.T @ c for c in cs)
    d = np.diag(dH).real
    X = np.stack([np.ones(256), np.diag(Nop)], 1)
    coef, *_ = np.linalg.lstsq(X, d, rcond=None)
    assert np.abs(dH - np.diag(X @ coef)).max() < 1e-12
    assert np.abs(Ho - Ho.conj().T).max() < 1e-12


def test_sphere_observables_fock_expectation():
    """Wick evaluation of S^i_{l,m} on the sphere equals Tr[B n n^+]/Tr B in Fock
    space for (l, m) = (0, 0), (1, 0), (1, 1); m^2_SO(5) uses (l, m) = (0, 0)."""
    n, L = 2, 2
    m = Model(n, L, 0.1, u0=1.0, uk=1.0, un=1.0, q_mode=Q_SPHERE)
    cs = fock.annihilators(4 * n)
    Qops = [fock.component_operators_sphere(cs, n, m.comps, PAULI[i], i == 0) for i in range(4)]
    phi = synth.fields(72, L, m.n_q)
    Bf = np.eye(256, dtype=complex)
    for t in range(L):
        Bt = np.eye(256, dtype=complex)
        for i in range(4):
            Bt = Bt @ sla.expm(m.alpha[i] * sum(phi[t, i, c] * Qops[i][c] for c in range(m.n_q)))
        Bf = Bt @ Bf
    G = dqmc.green(m, phi, L)
    for gm in gamma_matrices():
        for (l, mm) in [(0, 0), (1, 0), (1, 1)]:
            a = fock.density_operator_sphere(cs, n, l, mm, gm, False)
            ex = np.trace(Bf @ a @ a.conj().T) / np.trace(Bf)
            assert abs(ex - structure_factor(G, n, gm, l, mm, sphere=True)) < 1e-11
    s, m2 = so5_observables(G, n, sphere=True)
    assert abs(s[2] - s[3]) < 1e-12 and abs(s[3] - s[4]) < 1e-12
    assert abs(m2 - s.real.sum() / (5 * n * n)) < 1e-15


def test_sphere_sign_free_and_half_filling():
    """Random fields on the sphere (N = 3, 4): ln w is real mod 2 pi i and
    Re tr G_4N = 2N (particle-hole symmetry at half filling)."""
    for n in (3, 4):
        m = Model(n, 6, 0.1, u0=1.0, uk=1.5, un=1.5, q_mode=Q_SPHERE)
        phi = synth.fields(73 + n, 6, m.n_q)
        ld = dqmc.logdet(m, phi)
        assert abs(np.angle(np.exp(1j * ld.imag))) < 1e-9
        G = dqmc.green(m, phi, 0)
        assert abs(2 * np.trace(G).real - 2 * n) < 1e-10

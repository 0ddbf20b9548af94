"""Spherical regularisation of the projected model (oracle side, FP64).

Methods, "Spherical regularization": Dirac fermions on a sphere around a
monopole of charge 4 pi s; the lowest Landau level has N = 2s + 1 orbitals
with L_z eigenvalue m_k = k - 1 - s (k = 1..N, monopole harmonics), and the
density operator of angular momentum (l, m), 0 <= l <= 2s, is a sum over
orbitals of Wigner 3j weights (eq. sphere density operator).

Readings (see the design notes):
  * the printed k inside the 3j symbol and in the sign is the orbital's m_k
    (the 3j symbol needs -s <= -k <= s): the weight of c^dagger_k c_{k'} with
    m_{k'} = m_k + m is (-1)^(s + m_k + m) (2s+1) sqrt(2l+1) / 2
    * 3j(s l s; -m_k, -m, m_k + m) * 3j(s l s; -s, 0, s);
  * every (l, m) with l <= 2s enters (the 3j symbols vanish for l > 2s), N^2
    momenta per channel;
  * the pair n_q n_{-q} of the interaction is n_{l,m} n_{l,m}^dagger, so the
    Hermitian HS components per channel are sqrt(2) n_{l,0} (l = 0..2s) and,
    for 0 < m <= l, n_{l,m} + n_{l,m}^dagger and i (n_{l,m} - n_{l,m}^dagger);
    ordered by m, then l (A before C);
  * the background -2 per orbital applies to O^0 and m = 0 (every l), as a
    c-number -2 tr(n_{l,0}).
"""
import math
from fractions import Fraction

import numpy as np


def wigner3j(tj1, tj2, tj3, tm1, tm2, tm3):
    """Wigner 3j symbol (j1 j2 j3; m1 m2 m3) from doubled integer arguments
    (2j, 2m), by Racah's single-sum formula in exact rational arithmetic
    (Edmonds, Angular Momentum in Quantum Mechanics, eq. 3.7.3)."""
    if tm1 + tm2 + tm3 != 0:
        return 0.0
    for tj, tm in ((tj1, tm1), (tj2, tm2), (tj3, tm3)):
        if abs(tm) > tj or (tj + tm) % 2:
            return 0.0
    if tj3 < abs(tj1 - tj2) or tj3 > tj1 + tj2 or (tj1 + tj2 + tj3) % 2:
        return 0.0
    f = math.factorial
    a = (tj1 + tj2 - tj3) // 2
    b = (tj1 - tj2 + tj3) // 2
    c = (-tj1 + tj2 + tj3) // 2
    d = (tj1 + tj2 + tj3) // 2 + 1
    tri = Fraction(f(a) * f(b) * f(c), f(d))
    pre = (f((tj1 + tm1) // 2) * f((tj1 - tm1) // 2) * f((tj2 + tm2) // 2) * f((tj2 - tm2) // 2)
           * f((tj3 + tm3) // 2) * f((tj3 - tm3) // 2))
    # k ranges over values keeping every factorial argument non-negative
    x1 = (tj3 - tj2 + tm1) // 2
    x2 = (tj3 - tj1 - tm2) // 2
    x3 = (tj1 + tj2 - tj3) // 2
    x4 = (tj1 - tm1) // 2
    x5 = (tj2 + tm2) // 2
    s = Fraction(0)
    for k in range(max(0, -x1, -x2), min(x3, x4, x5) + 1):
        den = f(k) * f(x1 + k) * f(x2 + k) * f(x3 - k) * f(x4 - k) * f(x5 - k)
        s += Fraction((-1) ** k, den)
    if s == 0:
        return 0.0
    sign = -1 if ((tj1 - tj2 - tm3) // 2) % 2 else 1
    if s < 0:
        sign = -sign
    # the square tri * pre * s^2 is a rational of moderate size (|3j| <= 1)
    # even where tri * pre alone exceeds the float range
    return sign * math.sqrt(float(tri * pre * s * s))


def orbital_m2(n_phi):
    """Doubled L_z eigenvalues 2 m_k = 2(k - 1 - s) = 2k - 2 - (N - 1), k = 1..N."""
    return [2 * (k - 1) - (n_phi - 1) for k in range(1, n_phi + 1)]


def density_matrix(l, m, n_phi):
    """Orbital matrix of n_{l,m} (eq. sphere density operator, reading above):
    entry [k-1, k'-1] for m_{k'} = m_k + m."""
    ts = n_phi - 1                       # 2s
    mk2 = orbital_m2(n_phi)
    out = np.zeros((n_phi, n_phi), dtype=complex)
    if l > ts:
        return out
    norm = (ts + 1) * math.sqrt(2 * l + 1) / 2.0 * wigner3j(ts, 2 * l, ts, -ts, 0, ts)
    for r in range(n_phi):
        c = r + m
        if c < 0 or c >= n_phi:
            continue
        # (-1)^(s + m_k + m) with s + m_k = k - 1 = r
        sign = -1.0 if (r + m) % 2 else 1.0
        out[r, c] = sign * norm * wigner3j(ts, 2 * l, ts, -mk2[r], -2 * m, mk2[r] + 2 * m)
    return out


def momenta(n_phi):
    """All (l, m) with 0 <= l <= 2s, -l <= m <= l."""
    return [(l, m) for l in range(n_phi) for m in range(-l, l + 1)]


def components(n_phi):
    """Real HS components of one channel: ('S', l, 0) for every l, then for
    each m = 1..2s and l = m..2s the pair ('A', l, m), ('C', l, m)."""
    comps = [('S', l, 0) for l in range(n_phi)]
    for m in range(1, n_phi):
        for l in range(m, n_phi):
            comps.append(('A', l, m))
            comps.append(('C', l, m))
    return comps


def component_matrix(kind, l, m, n_phi):
    a = density_matrix(l, m, n_phi)
    if kind == 'S':
        return np.sqrt(2.0) * a
    if kind == 'A':
        return a + a.conj().T
    if kind == 'C':
        return 1j * (a - a.conj().T)
    raise ValueError(kind)


def lz_lplus(n_phi):
    """One-body L_z and L_+ on the LLL orbitals (m_k = k - 1 - s):
    L_+ |m> = sqrt((s - m)(s + m + 1)) |m + 1>."""
    ts = n_phi - 1
    mk2 = orbital_m2(n_phi)
    lz = np.diag([x / 2.0 for x in mk2]).astype(complex)
    lp = np.zeros((n_phi, n_phi), dtype=complex)
    for r in range(n_phi - 1):
        m = mk2[r] / 2.0
        lp[r + 1, r] = math.sqrt((ts / 2.0 - m) * (ts / 2.0 + m + 1))
    return lz, lp


def monopole_harmonic(k, n_phi, theta, phi):
    """LLL wave function of orbital k (Methods): N_m e^{i m phi}
    cos^{s+m}(theta/2) sin^{s-m}(theta/2), m = k - 1 - s."""
    s = (n_phi - 1) / 2.0
    m = k - 1 - s
    nrm = math.sqrt(math.factorial(n_phi) / (4.0 * math.pi * math.factorial(int(round(s + m)))
                                             * math.factorial(int(round(s - m)))))
    return nrm * np.exp(1j * m * phi) * np.cos(theta / 2) ** (s + m) * np.sin(theta / 2) ** (s - m)

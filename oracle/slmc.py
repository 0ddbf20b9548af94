"""Self-learning proposal (SLMC) for the continuous-field sweep: FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper's Methods section samples the HS fields with whole-slice Langevin
moves (eq. Langevin proposal) under the Metropolis-Hastings test. The learned
proposal adds global moves in the spirit of self-learning Monte Carlo: an
effective bosonic action S_eff(phi) = |phi|^2 / 2 + S_NN(phi) is fitted to the
exact weight, a Markov chain that is reversible for exp(-S_eff) (here Hybrid
Monte Carlo with its own accept step) proposes phi', and the exact weight
decides

    ln A = ln w_F(phi') - ln w_F(phi) + S_NN(phi') - S_NN(phi),

with w_F the fermion weight of the partition function (eq. HS transform and
the determinant form of Z). The Gaussian part of the true action cancels
against the Gaussian part of S_eff.

S_NN is a three-layer perceptron on symmetry-reduced features of phi:
  * the periodogram of every field component along imaginary time,
    P^i_c(w) = |sum_tau phi^i_{tau,c} exp(-2 pi i w tau / L)|^2 / L,
    w = 0..L/2, averaged over bins of (channel i, |q|^2 shell of c, w range);
  * the imaginary-time mean of the q = 0 component of every channel,
    sum_tau phi^i_{tau,0} / sqrt(L).
Both are invariant under cyclic translation in tau, a symmetry of the weight.
The network is tanh(W1 x + b1) -> tanh(W2 . + b2) -> w3 . + b3 on the
standardised features x = (f - mu) / sigma, with output s_y * out + y_bar.

BF16 rounding points (bf16=True) mirror the GPU kernels: every operand of a
matrix product (weights, layer inputs, back-propagated deltas) is rounded to
bfloat16 (round to nearest even) and products accumulate in higher precision.
With bf16=False the same code is the exact FP64 function (finite-difference
pins apply to it).

Parity: pinned by Parseval's identity, translation invariance, finite
differences of the exact path, torch's bfloat16 conversion and Adam
optimiser (library routines), leapfrog reversibility and energy error, and
the stationary law of the global-move chain on a Gaussian target.
"""
import numpy as np

from .model import Model


# ------------------------------------------------------------------ features

def component_shells(model: Model, n_qbins):
    """Shell index of every HS component: s = floor(n_qbins r2 / (r2_max + 1))
    with r2 = qx^2 + qy^2 of the component's momentum (integer arithmetic)."""
    r2 = np.array([qx * qx + qy * qy for (_, qx, qy) in model.comps], dtype=np.int64)
    return (n_qbins * r2) // (r2.max() + 1)


def freq_bins(l_tau, n_wbins):
    """Bin of every frequency w = 0..L/2: floor(n_wbins w / (L/2 + 1))."""
    nw = l_tau // 2 + 1
    return (n_wbins * np.arange(nw)) // nw


class FeatureMap:
    def __init__(self, model: Model, n_qbins, n_wbins):
        self.model, self.nqb, self.nwb = model, n_qbins, n_wbins
        self.L, self.nq = model.l_tau, model.n_q
        self.shell = component_shells(model, n_qbins)
        self.wbin = freq_bins(self.L, n_wbins)
        cs = np.bincount(self.shell, minlength=n_qbins)
        cw = np.bincount(self.wbin, minlength=n_wbins)
        self.count = np.outer(cs, cw)                  # members per (shell, w bin)
        self.n_feat = 4 * n_qbins * n_wbins + 4

    def dft(self, phi):
        """X^i_c(w) = sum_tau phi^i_{tau,c} exp(-2 pi i w tau / L), w = 0..L/2."""
        return np.fft.rfft(np.asarray(phi, dtype=float), axis=0)      # [nw][4][nq]

    def features(self, phi):
        L = self.L
        X = self.dft(phi)
        P = np.abs(X) ** 2 / L                                         # [nw][4][nq]
        f = np.zeros((4, self.nqb, self.nwb))
        for i in range(4):
            S = np.zeros((self.nqb, self.nwb))
            np.add.at(S, (self.shell[None, :], self.wbin[:, None]), P[:, i, :])
            f[i] = np.where(self.count > 0, S / np.maximum(self.count, 1), 0.0)
        lin = np.asarray(phi, dtype=float)[:, :, 0].sum(axis=0) / np.sqrt(L)
        return np.concatenate([f.reshape(-1), lin])

    def features_vjp(self, phi, g):
        """d(g . f(phi)) / d phi for a feature cotangent g [n_feat]."""
        L = self.L
        X = self.dft(phi)                                              # [nw][4][nq]
        gb = g[:-4].reshape(4, self.nqb, self.nwb)
        coef = np.where(self.count > 0, 1.0 / np.maximum(self.count, 1), 0.0)
        # gamma^i_c(w) = g[i, s(c), w(w)] / count ; dP/dphi_tau = (2/L) Re[conj(X) e^{-2 pi i w tau/L}]
        gam = (gb * coef[None])[:, self.shell[:, None], self.wbin[None, :]]     # [4][nq][nw]
        tau = np.arange(L)
        w = np.arange(X.shape[0])
        ph = np.exp(-2j * np.pi * np.outer(tau, w) / L)                # [L][nw]
        Y = np.conj(X).transpose(1, 2, 0) * gam                        # [4][nq][nw]
        out = (2.0 / L) * np.real(np.einsum('icw,tw->tic', Y, ph))
        out[:, :, 0] += g[-4:][None, :] / np.sqrt(L)
        return out


# ------------------------------------------------------------------ BF16

def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    Works on the float32 bit pattern: add 0x7FFF plus the lowest kept bit,
    then clear the low 16 bits (inputs are finite)."""
    a = np.asarray(x, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


# ------------------------------------------------------------------ MLP

class MLP:
    """Parameters in the flat order W1 [H][F], b1 [H], W2 [H][H], b2 [H],
    w3 [H], b3 [1]."""

    def __init__(self, n_feat, hidden, rng=None, params=None):
        self.F, self.H = n_feat, hidden
        if params is not None:
            self.set_flat(params)
        else:
            rng = rng or np.random.default_rng(0)
            self.W1 = rng.normal(size=(hidden, n_feat)) / np.sqrt(n_feat)
            self.b1 = np.zeros(hidden)
            self.W2 = rng.normal(size=(hidden, hidden)) / np.sqrt(hidden)
            self.b2 = np.zeros(hidden)
            self.w3 = rng.normal(size=hidden) / np.sqrt(hidden)
            self.b3 = np.zeros(1)
        self.mu = np.zeros(n_feat)
        self.sigma = np.ones(n_feat)
        self.y_bar, self.s_y = 0.0, 1.0

    def n_params(self):
        F, H = self.F, self.H
        return H * F + H + H * H + H + H + 1

    def flat(self):
        return np.concatenate([self.W1.ravel(), self.b1, self.W2.ravel(), self.b2, self.w3, self.b3])

    def set_flat(self, p):
        F, H = self.F, self.H
        p = np.asarray(p, dtype=float)
        o = 0
        self.W1 = p[o:o + H * F].reshape(H, F); o += H * F
        self.b1 = p[o:o + H].copy(); o += H
        self.W2 = p[o:o + H * H].reshape(H, H); o += H * H
        self.b2 = p[o:o + H].copy(); o += H
        self.w3 = p[o:o + H].copy(); o += H
        self.b3 = p[o:o + 1].copy()

    def fit_norm(self, feats, y):
        """Standardisation of features and target from a data set."""
        self.mu = feats.mean(axis=0)
        sd = feats.std(axis=0)
        self.sigma = np.where(sd > 1e-12, sd, 1.0)
        self.y_bar = float(np.mean(y))
        sy = float(np.std(y))
        self.s_y = sy if sy > 1e-12 else 1.0

    def forward(self, x, bf16=False):
        """x [B][F] standardised features -> out [B] and the saved activations."""
        r = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=float))
        xr = r(x)
        a1 = np.tanh(xr @ r(self.W1).T + self.b1)
        a1r = r(a1)
        a2 = np.tanh(a1r @ r(self.W2).T + self.b2)
        a2r = r(a2)
        out = a2r @ r(self.w3) + self.b3[0]
        return out, (xr, a1, a1r, a2, a2r)

    def backward(self, dout, cache, bf16=False):
        """Gradients of sum_b dout[b] out[b] w.r.t. the parameters and x."""
        r = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=float))
        xr, a1, a1r, a2, a2r = cache
        dout = np.asarray(dout, dtype=float)
        g = {}
        g['w3'] = a2r.T @ dout
        g['b3'] = np.array([dout.sum()])
        dz2 = np.outer(dout, r(self.w3)) * (1.0 - a2 ** 2)
        dz2r = r(dz2)
        g['W2'] = dz2r.T @ a1r
        g['b2'] = dz2.sum(axis=0)
        dz1 = (dz2r @ r(self.W2)) * (1.0 - a1 ** 2)
        dz1r = r(dz1)
        g['W1'] = dz1r.T @ xr
        g['b1'] = dz1.sum(axis=0)
        dx = dz1r @ r(self.W1)
        flat = np.concatenate([g['W1'].ravel(), g['b1'], g['W2'].ravel(), g['b2'], g['w3'], g['b3']])
        return flat, dx

    def loss_grad(self, x, y_std, bf16=False):
        """Mean squared error against standardised targets and its gradient."""
        out, cache = self.forward(x, bf16)
        B = len(y_std)
        res = out - y_std
        loss = float(np.mean(res ** 2))
        gflat, _ = self.backward(2.0 * res / B, cache, bf16)
        return loss, gflat

    def action(self, fmap: FeatureMap, phis, bf16=False):
        """S_NN(phi) = s_y out((f - mu) / sigma) + y_bar for a list of configurations."""
        f = np.stack([fmap.features(p) for p in phis])
        x = (f - self.mu) / self.sigma
        out, _ = self.forward(x, bf16)
        return self.s_y * out + self.y_bar

    def action_grad(self, fmap: FeatureMap, phi, bf16=False):
        """S_NN(phi) and dS_NN/dphi for one configuration [L][4][nq]."""
        f = fmap.features(phi)
        x = ((f - self.mu) / self.sigma)[None]
        out, cache = self.forward(x, bf16)
        _, dx = self.backward(np.array([self.s_y]), cache, bf16)
        gf = dx[0] / self.sigma
        return self.s_y * out[0] + self.y_bar, fmap.features_vjp(phi, gf)


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), t = step number starting at 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ HMC and the global move

def hmc_trajectory_uniform(phi, p0, grad_s, s_eff, step, n_leap):
    """Leapfrog for H = S_eff + |p|^2 / 2 in the four coordinates
    A_i = sum_tau phi^i_{tau,0} / sqrt(L) of fields [L][4][n_q] (every slice's
    component 0 shifted together); p0 holds their momenta at [0][i][0], the
    force on A_i is sum_tau dS_eff/dphi^i_{tau,0} / sqrt(L). Returns (phi', dH)."""
    q = np.array(phi, dtype=float)
    L = q.shape[0]
    r = 1.0 / np.sqrt(L)
    p = np.array(p0, dtype=float)[0, :, 0].copy()
    force = lambda x: grad_s(x)[:, :, 0].sum(axis=0) * r
    h0 = s_eff(q) + 0.5 * np.sum(p * p)
    p = p - 0.5 * step * force(q)
    for k in range(n_leap):
        q[:, :, 0] += step * p * r
        if k < n_leap - 1:
            p = p - step * force(q)
    p = p - 0.5 * step * force(q)
    h1 = s_eff(q) + 0.5 * np.sum(p * p)
    return q, h1 - h0


def hmc_trajectory(phi, p0, grad_s, s_eff, step, n_leap, mask=None):
    """Leapfrog trajectory for H = S_eff(phi) + |p|^2 / 2. Returns (phi', dH).
    mask (same shape as phi, 0/1): only the coordinates with mask 1 carry
    momentum and move; the rest stay fixed (HMC on the conditional of the
    masked coordinates, still reversible for exp(-S_eff)). mask = "uniform":
    the four slice-uniform q = 0 amplitudes (hmc_trajectory_uniform)."""
    if isinstance(mask, str):
        return hmc_trajectory_uniform(phi, p0, grad_s, s_eff, step, n_leap)
    q = np.array(phi, dtype=float)
    p = np.array(p0, dtype=float)
    m = np.ones_like(q) if mask is None else np.asarray(mask, dtype=float)
    p = p * m
    h0 = s_eff(q) + 0.5 * np.sum(p * p)
    p = p - 0.5 * step * grad_s(q) * m
    for k in range(n_leap):
        q = q + step * p
        if k < n_leap - 1:
            p = p - step * grad_s(q) * m
    p = p - 0.5 * step * grad_s(q) * m
    h1 = s_eff(q) + 0.5 * np.sum(p * p)
    return q, h1 - h0


def q0_mask(shape):
    """Mask of component 0 (q = 0) of every channel and slice for fields of
    shape [L][4][n_q]."""
    m = np.zeros(shape)
    m[..., 0] = 1.0
    return m


def inner_chain(phi, momenta, uniforms, grad_s, s_eff, step, n_leap, mask=None):
    """HMC trajectories with their own Metropolis test (reversible for
    exp(-S_eff)); momenta [n_traj][...] and uniforms [n_traj] are inputs."""
    q = np.array(phi, dtype=float)
    acc = 0
    for p0, u in zip(momenta, uniforms):
        qn, dh = hmc_trajectory(q, p0, grad_s, s_eff, step, n_leap, mask)
        if np.log(u) < -dh:
            q, acc = qn, acc + 1
    return q, acc


def global_move_lnA(lnw, lnw_new, s_nn, s_nn_new):
    """ln A of the learned global move (see the module header)."""
    return (lnw_new - lnw) + (s_nn_new - s_nn)

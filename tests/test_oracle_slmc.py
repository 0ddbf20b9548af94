"""Pins of the SLMC oracle (features, network, optimiser, HMC, global move)."""
import numpy as np
import pytest

from oracle.model import Model, Q_BZ, Q_PAPER
from oracle import slmc


def _fmap(n_phi=6, L=20, nqb=4, nwb=5, mode=Q_BZ):
    m = Model(n_phi, L, 0.1, u0=1.0, uk=1.0, un=1.0, q_mode=mode)
    return m, slmc.FeatureMap(m, nqb, nwb)


def test_periodogram_parseval():
    """One-sided periodogram sums back to sum_tau phi^2 (Parseval), odd and even L."""
    for L in (20, 21):
        m, fm = _fmap(L=L)
        phi = np.random.default_rng(1).normal(size=(L, 4, m.n_q))
        P = np.abs(fm.dft(phi)) ** 2 / L
        w = np.full(P.shape[0], 2.0)
        w[0] = 1.0
        if L % 2 == 0:
            w[-1] = 1.0
        assert np.allclose(np.einsum('w,wic->ic', w, P), (phi ** 2).sum(axis=0), rtol=1e-12)


def test_features_of_a_single_cosine():
    """phi = cos(2 pi w0 tau / L) on one component: P(w0) = L / 4, all else 0."""
    m, fm = _fmap(L=24)
    L, w0, i, c = 24, 5, 2, 7
    phi = np.zeros((L, 4, m.n_q))
    phi[:, i, c] = np.cos(2 * np.pi * w0 * np.arange(L) / L)
    f = fm.features(phi)
    ref = np.zeros((4, fm.nqb, fm.nwb))
    s, wb = fm.shell[c], fm.wbin[w0]
    ref[i, s, wb] = (L / 4.0) / fm.count[s, wb]
    assert np.allclose(f[:-4], ref.ravel(), atol=1e-12)
    assert np.allclose(f[-4:], 0.0, atol=1e-12)


def test_shells_and_bins_partition():
    m, fm = _fmap(n_phi=7, L=30, nqb=6, nwb=7, mode=Q_PAPER)
    assert fm.shell[0] == 0 and fm.shell.max() == fm.nqb - 1
    assert fm.wbin[0] == 0 and fm.wbin[-1] == fm.nwb - 1
    assert fm.count.sum() == m.n_q * (30 // 2 + 1)


def test_features_translation_invariant():
    m, fm = _fmap()
    phi = np.random.default_rng(2).normal(size=(20, 4, m.n_q))
    assert np.allclose(fm.features(np.roll(phi, 7, axis=0)), fm.features(phi), rtol=1e-12, atol=1e-12)


def test_feature_vjp_finite_differences():
    m, fm = _fmap(L=9)
    rng = np.random.default_rng(3)
    phi = rng.normal(size=(9, 4, m.n_q))
    g = rng.normal(size=fm.n_feat)
    grad = fm.features_vjp(phi, g)
    h = 1e-6
    for (t, i, c) in [(0, 0, 0), (3, 1, 2), (8, 3, m.n_q - 1), (4, 2, 5), (5, 0, 0)]:
        d = np.zeros_like(phi)
        d[t, i, c] = h
        fd = (g @ fm.features(phi + d) - g @ fm.features(phi - d)) / (2 * h)
        assert abs(fd - grad[t, i, c]) < 1e-7 * max(1.0, abs(fd))


def test_mlp_backward_finite_differences():
    rng = np.random.default_rng(4)
    net = slmc.MLP(11, 7, rng)
    net.b1 = rng.normal(size=7) * 0.1
    x = rng.normal(size=(5, 11))
    y = rng.normal(size=5)
    loss, g = net.loss_grad(x, y)
    p0 = net.flat()
    h = 1e-6
    for k in rng.choice(len(p0), 25, replace=False).tolist() + [len(p0) - 1]:
        d = np.zeros_like(p0)
        d[k] = h
        net.set_flat(p0 + d)
        lp, _ = net.loss_grad(x, y)
        net.set_flat(p0 - d)
        lm, _ = net.loss_grad(x, y)
        net.set_flat(p0)
        assert abs((lp - lm) / (2 * h) - g[k]) < 1e-7 * max(1.0, abs(g[k]))
    # input gradient
    out, cache = net.forward(x)
    dout = rng.normal(size=5)
    _, dx = net.backward(dout, cache)
    for (b, j) in [(0, 0), (2, 5), (4, 10)]:
        d = np.zeros_like(x)
        d[b, j] = h
        fd = (dout @ net.forward(x + d)[0] - dout @ net.forward(x - d)[0]) / (2 * h)
        assert abs(fd - dx[b, j]) < 1e-7


def test_action_gradient_finite_differences():
    m, fm = _fmap(L=10)
    rng = np.random.default_rng(5)
    net = slmc.MLP(fm.n_feat, 9, rng)
    phis = [rng.normal(size=(10, 4, m.n_q)) for _ in range(6)]
    net.fit_norm(np.stack([fm.features(p) for p in phis]), rng.normal(size=6) * 3 + 1)
    phi = phis[0]
    s, g = net.action_grad(fm, phi)
    assert abs(s - net.action(fm, [phi])[0]) < 1e-12
    h = 1e-6
    for (t, i, c) in [(0, 0, 0), (2, 1, 3), (9, 3, m.n_q - 1), (6, 2, 1)]:
        d = np.zeros_like(phi)
        d[t, i, c] = h
        fd = (net.action(fm, [phi + d])[0] - net.action(fm, [phi - d])[0]) / (2 * h)
        assert abs(fd - g[t, i, c]) < 1e-6 * max(1.0, abs(fd))


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    x = np.concatenate([rng.normal(size=4000) * 10.0 ** rng.integers(-8, 8, 4000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, -3.0e-39]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(slmc.bf16_round(x), ref)


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    p = rng.normal(size=30)
    grads = [rng.normal(size=30) for _ in range(4)]
    tp = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=3e-3)
    m = np.zeros(30)
    v = np.zeros(30)
    q = p.copy()
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
        q, m, v = slmc.adam_step(q, g, m, v, t, 3e-3)
    assert np.allclose(q, tp.detach().numpy(), rtol=0, atol=1e-14)


def _quartic():
    s = lambda q: 0.5 * np.sum(q * q) + 0.05 * np.sum(q ** 4)
    g = lambda q: q + 0.2 * q ** 3
    return s, g


def test_leapfrog_reversible_and_second_order():
    s, g = _quartic()
    rng = np.random.default_rng(8)
    q0 = rng.normal(size=50)
    p0 = rng.normal(size=50)
    q1, _ = slmc.hmc_trajectory(q0, p0, g, s, 0.1, 12)
    # momentum at the end, flipped, brings the trajectory back
    p = p0 - 0.05 * g(q0)
    q = q0.copy()
    for k in range(12):
        q = q + 0.1 * p
        p = p - (0.1 if k < 11 else 0.05) * g(q)
    qb, _ = slmc.hmc_trajectory(q1, -p, g, s, 0.1, 12)
    assert np.abs(qb - q0).max() < 1e-12
    dh = [abs(slmc.hmc_trajectory(q0, p0, g, s, h, int(round(1.2 / h)))[1]) for h in (0.1, 0.05)]
    assert 3.0 < dh[0] / dh[1] < 5.0


def test_global_move_chain_samples_the_exact_law():
    """Gaussian target exp(-(1 + a)|phi|^2 / 2) with the 'fermion' part
    ln w = -a |phi|^2 / 2 and a deliberately wrong model S_NN = b |phi|^2 / 2:
    HMC proposals on S_eff plus the global test must still give variance
    1 / (1 + a), not the model's 1 / (1 + b)."""
    a, b, d = 0.5, 0.25, 8
    lnw = lambda q: -0.5 * a * np.sum(q * q)
    snn = lambda q: 0.5 * b * np.sum(q * q)
    s_eff = lambda q: 0.5 * np.sum(q * q) + snn(q)
    g_eff = lambda q: (1.0 + b) * q
    rng = np.random.default_rng(9)
    q = rng.normal(size=d)
    acc, samples = 0, []
    for it in range(6000):
        qn, _ = slmc.inner_chain(q, rng.normal(size=(1, d)), rng.random(1), g_eff, s_eff, 0.3, 5)
        la = slmc.global_move_lnA(lnw(q), lnw(qn), snn(q), snn(qn))
        if np.log(rng.random()) < la:
            q, acc = qn, acc + 1
        samples.append(q.copy())
    x = np.array(samples[500:])
    assert 0.2 < acc / 6000 < 0.99
    assert abs(x.var() - 1.0 / (1.0 + a)) < 0.04
    assert abs(x.var() - 1.0 / (1.0 + b)) > 0.08


def test_masked_global_move_moves_only_its_subspace_and_samples_its_law():
    """With a mask (the q = 0 subspace of the learned move) the unmasked
    coordinates never change and the masked ones sample the exact conditional
    law 1 / (1 + a), not the model's 1 / (1 + b); the masked leapfrog is still
    reversible."""
    a, b = 0.5, 0.25
    shape = (6, 4, 3)                      # [L][4][n_q]
    mask = slmc.q0_mask(shape)
    assert mask.sum() == 24 and np.all(mask[..., 1:] == 0)
    lnw = lambda q: -0.5 * a * np.sum(q * q)
    snn = lambda q: 0.5 * b * np.sum(q * q)
    s_eff = lambda q: 0.5 * np.sum(q * q) + snn(q)
    g_eff = lambda q: (1.0 + b) * q
    rng = np.random.default_rng(10)
    q = rng.normal(size=shape)
    fixed = q[..., 1:].copy()
    p0 = rng.normal(size=shape)
    q1, _ = slmc.hmc_trajectory(q, p0, g_eff, s_eff, 0.2, 6, mask)
    assert np.array_equal(q1[..., 1:], fixed)
    # reverse: end momentum flipped returns to the start (masked leapfrog)
    p = p0 * mask - 0.1 * g_eff(q) * mask
    qq = q.copy()
    for k in range(6):
        qq = qq + 0.2 * p
        p = p - (0.2 if k < 5 else 0.1) * g_eff(qq) * mask
    qb, _ = slmc.hmc_trajectory(q1, -p, g_eff, s_eff, 0.2, 6, mask)
    assert np.abs(qb - q).max() < 1e-12
    acc, samples = 0, []
    for it in range(4000):
        qn, _ = slmc.inner_chain(q, rng.normal(size=(1,) + shape), rng.random(1), g_eff, s_eff, 0.3, 5, mask)
        la = slmc.global_move_lnA(lnw(q), lnw(qn), snn(q), snn(qn))
        if np.log(rng.random()) < la:
            q, acc = qn, acc + 1
        samples.append(q[..., 0].copy())
    assert np.array_equal(q[..., 1:], fixed)
    x = np.array(samples[300:])
    assert 0.2 < acc / 4000 < 0.99
    assert abs(x.var() - 1.0 / (1.0 + a)) < 0.04


def test_uniform_mode_global_move_shifts_all_slices_together_and_samples_its_law():
    """The slice-uniform q = 0 subspace: every slice's component 0 moves by the
    same amount, everything else stays, the leapfrog is reversible, and on a
    Gaussian target the amplitude A_i = sum_tau phi / sqrt(L) samples its exact
    conditional law 1 / (1 + a) (the model says 1 / (1 + b))."""
    a, b = 0.5, 0.25
    shape = (6, 4, 3)
    lnw = lambda q: -0.5 * a * np.sum(q * q)
    snn = lambda q: 0.5 * b * np.sum(q * q)
    s_eff = lambda q: 0.5 * np.sum(q * q) + snn(q)
    g_eff = lambda q: (1.0 + b) * q
    rng = np.random.default_rng(12)
    q = rng.normal(size=shape)
    p0 = rng.normal(size=shape)
    q1, _ = slmc.hmc_trajectory(q, p0, g_eff, s_eff, 0.3, 5, "uniform")
    d = q1[:, :, 0] - q[:, :, 0]
    assert np.abs(d - d[0]).max() < 1e-14 and np.abs(d[0]).max() > 1e-3
    assert np.array_equal(q1[..., 1:], q[..., 1:])
    # reversibility: rerun from the end with the flipped final momentum of A
    L = shape[0]
    force = lambda x: g_eff(x)[:, :, 0].sum(axis=0) / np.sqrt(L)
    p = p0[0, :, 0] - 0.15 * force(q)
    qq = q.copy()
    for k in range(5):
        qq[:, :, 0] += 0.3 * p / np.sqrt(L)
        p = p - (0.3 if k < 4 else 0.15) * force(qq)
    pb = np.zeros(shape)
    pb[0, :, 0] = -p
    qb, _ = slmc.hmc_trajectory(q1, pb, g_eff, s_eff, 0.3, 5, "uniform")
    assert np.abs(qb - q).max() < 1e-12
    centred = q[:, :, 0] - q[:, :, 0].mean(axis=0)
    fixed = q[..., 1:].copy()
    samples, acc = [], 0
    for it in range(4000):
        qn, _ = slmc.inner_chain(q, rng.normal(size=(1,) + shape), rng.random(1), g_eff, s_eff, 0.4, 4, "uniform")
        la = slmc.global_move_lnA(lnw(q), lnw(qn), snn(q), snn(qn))
        if np.log(rng.random()) < la:
            q, acc = qn, acc + 1
        samples.append(q[:, :, 0].sum(axis=0) / np.sqrt(L))
    assert np.array_equal(q[..., 1:], fixed)
    assert np.abs(q[:, :, 0] - q[:, :, 0].mean(axis=0) - centred).max() < 1e-12
    x = np.array(samples[300:])
    assert 0.2 < acc / 4000 < 0.99
    assert abs(x.var() - 1.0 / (1.0 + a)) < 0.05

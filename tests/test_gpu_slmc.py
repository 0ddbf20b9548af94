"""GPU parity of the learned global proposal against the SLMC oracle.

Tolerances: features are summed in FP32 (relative 1e-5). The network rounds
every product operand to BF16 (8-bit mantissa) exactly where the oracle's
bf16=True path does, so GPU and oracle differ only by FP32 vs FP64
accumulation and by the rare operand that lands on the other side of a BF16
rounding boundary (one BF16 ulp, 2^-8 relative, diluted over the H or F terms
of a product): relative 1e-2 on gradients and 2e-3 of s_y on S_NN. The exact
weights ln w_F of the global test are FP64 from scratch (1e-10).
"""
import numpy as np
import pytest

import synth
from oracle import dqmc, slmc
from oracle.model import Model, Q_BZ

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_03700_amd import CFQMC, Slmc
    return CFQMC, Slmc


def relmax(a, b):
    return np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(b).max(), 1e-300)


def _setup(n_phi=6, L=20, u=1.5, nch=2, hidden=32, nqb=4, nwb=5, seed=3):
    CFQMC, Slmc = _gpu()
    m = Model(n_phi, L, 0.1, u0=1.0, uk=u, un=u, q_mode=Q_BZ)
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, u0=1.0, uk=u, un=u, q_mode=Q_BZ, n_stab=5, n_chains=nch,
              tile_cfg=1, seed=seed, eps0=0.4)
    s = Slmc(g, hidden=hidden, n_qbins=nqb, n_wbins=nwb, capacity=4096, max_batch=128, seed=seed)
    fm = slmc.FeatureMap(m, nqb, nwb)
    return m, g, s, fm


def _random_net(fm, hidden, rng, phis):
    net = slmc.MLP(fm.n_feat, hidden, rng)
    net.b1 = rng.normal(size=hidden) * 0.2
    net.b2 = rng.normal(size=hidden) * 0.2
    net.b3 = np.array([0.3])
    feats = np.stack([fm.features(p) for p in phis])
    net.fit_norm(feats, rng.normal(size=len(phis)) * 2.0 + 5.0)
    # the GPU holds FP32 master weights: use the FP32 values on both sides
    net.set_flat(np.float32(net.flat()).astype(np.float64))
    net.mu = np.float32(net.mu).astype(np.float64)
    net.sigma = np.float32(net.sigma).astype(np.float64)
    return net


def test_features_match_oracle():
    m, g, s, fm = _setup(L=21)
    phis = np.stack([synth.fields(40 + k, 21, m.n_q) for k in range(5)])
    f = s.features(phis)
    for k in range(5):
        ref = fm.features(phis[k])
        assert f.shape[1] == fm.n_feat
        assert relmax(f[k], ref) < 1e-5
    s.close()
    g.close()


def test_action_and_field_gradient_match_oracle():
    m, g, s, fm = _setup(hidden=48)
    rng = np.random.default_rng(11)
    phis = [synth.fields(60 + k, 20, m.n_q) for k in range(6)]
    net = _random_net(fm, 48, rng, phis)
    s.set_params(net.flat())
    s.set_norm(net.mu, net.sigma, net.y_bar, net.s_y)
    # the gradient-check entry point (cfqmc_slmc_grad_check) against the oracle
    S, G = s.grad_check(np.stack(phis))
    S2, G2 = s.action(np.stack(phis), grad=True)
    assert np.array_equal(S, S2) and np.array_equal(G, G2)
    for k, phi in enumerate(phis):
        sr, gr = net.action_grad(fm, phi, bf16=True)
        assert abs(S[k] - sr) < 2e-3 * net.s_y
        assert relmax(G[k], gr) < 1e-2
        # BF16 effect itself stays small against the exact FP64 network
        se, ge = net.action_grad(fm, phi, bf16=False)
        assert abs(S[k] - se) < 5e-2 * net.s_y and relmax(G[k], ge) < 1e-1
    s.close()
    g.close()


def test_loss_and_weight_gradients_match_oracle():
    m, g, s, fm = _setup(hidden=64, nqb=5, nwb=6)
    rng = np.random.default_rng(12)
    net = slmc.MLP(fm.n_feat, 64, rng)
    net.b1 = rng.normal(size=64) * 0.1
    net.set_flat(np.float32(net.flat()).astype(np.float64))
    s.set_params(net.flat())
    n = 37                                  # ragged against the 64-row tiles
    x = np.float32(rng.normal(size=(n, fm.n_feat))).astype(np.float64)
    y = rng.normal(size=n)
    loss, grad, out = s.loss_grad(x, y)
    lr_, gr = net.loss_grad(x, np.float32(y).astype(np.float64), bf16=True)
    assert abs(loss - lr_) < 1e-3 * lr_
    F, H = fm.n_feat, 64
    cuts = np.cumsum([0, H * F, H, H * H, H, H, 1])
    for a, b in zip(cuts[:-1], cuts[1:]):
        assert relmax(grad[a:b], gr[a:b]) < 1e-2, (a, b)
    s.close()
    g.close()


def test_training_step_is_adam_on_the_oracle_gradient():
    """Collect configurations from the sweep, one full-batch Adam step on the
    GPU, against the oracle's gradient (BF16 path) and Adam update."""
    m, g, s, fm = _setup(nch=4, hidden=32)
    g.init_fields(None)
    phis, lnw = [], []
    for k in range(6):
        g.sweep(1)
        s.collect()
        F_ = g.get_fields()
        for z in range(4):
            phis.append(F_[z])
            lnw.append(g.logdet(z).real)
            assert abs(lnw[-1] - dqmc.logdet(m, F_[z]).real) < 1e-9 * abs(lnw[-1])
    assert s.n_data() == 24
    p0 = s.get_params().astype(np.float64)
    s.train(epochs=1, batch=24, lr=1e-3, refit_norm=True)
    p1 = s.get_params().astype(np.float64)
    mu, sg, yb, sy = s.get_norm()
    feats = np.stack([fm.features(p) for p in phis])
    assert relmax(mu, feats.mean(axis=0)) < 1e-5
    y = -np.array(lnw)
    assert abs(yb - y.mean()) < 1e-9 * abs(y.mean()) and abs(sy - y.std()) < 1e-6 * y.std()
    net = slmc.MLP(fm.n_feat, 32, params=p0)
    x = (feats - mu.astype(np.float64)) / sg.astype(np.float64)
    _, gr = net.loss_grad(x, np.float32((y - yb) / sy).astype(np.float64), bf16=True)
    ref, _, _ = slmc.adam_step(p0, gr, np.zeros_like(p0), np.zeros_like(p0), 1, 1e-3)
    d = np.abs(p1 - ref)
    assert np.mean(d < 1e-5) > 0.99 and d.max() <= 2.01e-3
    s.close()
    g.close()


@pytest.mark.parametrize("sub", ["all", "q0", "uniform_q0"])
def test_global_move_replay_matches_oracle(sub):
    """A replayed global move (every field, or the q = 0 subspace only)
    reproduces the oracle's HMC trajectory, inner accept count, exact weight
    change, ln A and decision, and leaves the rebuilt state."""
    m, g, s, fm = _setup(nch=2, hidden=32, L=16)
    L, nq = 16, m.n_q
    g.init_fields(None)
    g.sweep(2)
    phi0 = g.get_fields()
    rng = np.random.default_rng(13)
    net = _random_net(fm, 32, rng, [phi0[0], phi0[1], synth.fields(1, L, nq)])
    net.W1 *= 0.3
    net.set_flat(np.float32(net.flat()).astype(np.float64))
    s.set_params(net.flat())
    s.set_norm(net.mu, net.sigma, net.y_bar, net.s_y)
    s.set_subspace(sub)
    n_traj, n_leap, step = 2, 4, 0.25
    nf = L * 4 * nq
    rp = np.empty((2, n_traj * nf + n_traj + 1))
    for z in range(2):
        rp[z, :n_traj * nf] = rng.normal(size=n_traj * nf)
        rp[z, n_traj * nf:] = [0.3, 0.6, 0.5]
    lw0 = [g.logdet(z).real for z in range(2)]
    moves = s.global_move(n_traj, n_leap, step, rp)
    for z in range(2):
        mv = moves[z]
        prop = s.last_proposal(z)
        # oracle inner chain from the same start and momenta (BF16-mirrored action)
        sf = lambda q: 0.5 * np.sum(q * q) + net.action_grad(fm, q, bf16=True)[0]
        gf = lambda q: q + net.action_grad(fm, q, bf16=True)[1]
        mom = rp[z, :n_traj * nf].reshape(n_traj, L, 4, nq)
        mask = {"all": None, "q0": slmc.q0_mask(phi0[z].shape), "uniform_q0": "uniform"}[sub]
        q, acc = slmc.inner_chain(phi0[z], mom, rp[z, n_traj * nf:n_traj * nf + n_traj], gf, sf, step, n_leap,
                                  mask)
        if sub != "all":
            assert np.array_equal(prop[..., 1:], phi0[z][..., 1:])
        if sub == "uniform_q0":
            d = prop[:, :, 0] - phi0[z][:, :, 0]
            assert np.abs(d - d[0]).max() < 1e-12          # every slice shifted by the same amount
        assert acc == mv["inner_accepted"]
        assert relmax(prop, q) < 1e-4
        # exact weight of the proposal (FP64 from scratch) and the test itself
        lw1 = dqmc.logdet(m, prop).real
        assert abs(mv["d_lnw"] - (lw1 - lw0[z])) < 1e-9 * abs(lw1)
        s_pair = s.action(np.stack([phi0[z], prop]))
        assert abs(mv["d_snn"] - (s_pair[1] - s_pair[0])) < 1e-9 * max(1.0, abs(s_pair[0]))
        assert abs(mv["ln_a"] - (mv["d_lnw"] + mv["d_snn"])) < 1e-12 * max(1.0, abs(mv["ln_a"]))
        assert mv["accepted"] == int(np.log(0.5) < mv["ln_a"])
        # state after the move: fields, weight and G rebuilt from scratch
        now = g.get_fields()[z]
        assert np.array_equal(now, prop if mv["accepted"] else phi0[z])
        assert abs(g.logdet(z).real - dqmc.logdet(m, now).real) < 1e-9 * abs(lw1)
        G = g.measure_G(z, L)[:2 * m.n_phi, :2 * m.n_phi]
        assert relmax(G, dqmc.green(m, now, L)) < 1e-10
    g.sweep(1)                              # the sweep continues from the rebuilt state
    s.close()
    g.close()


def test_trained_proposal_gains_over_untrained_and_gaussian():
    """Train S_NN on configurations of the plain sweep. On fresh configurations
    the trained network explains part of the variance of ln w_F, and the
    global-move acceptance with it beats the Gaussian proposal (network = 0)
    and the untrained network on the same chains."""
    CFQMC, Slmc = _gpu()
    n_phi, L, u, nch = 6, 40, 3.0, 16
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, u0=1.0, uk=u, un=u, q_mode=Q_BZ, n_stab=8, n_chains=nch,
              tile_cfg=1, seed=21, eps0=0.4)
    s = Slmc(g, hidden=32, n_qbins=12, n_wbins=L // 2 + 1, capacity=8192, max_batch=256, seed=5)
    g.init_fields(None)
    g.sweep(20)
    for k in range(150):
        g.sweep(1)
        s.collect()
    w_untrained = s.get_params()
    loss0 = s.train(epochs=1, batch=64, lr=1e-3, refit_norm=True)
    s.set_params(w_untrained)
    loss = s.train(epochs=20, batch=64, lr=1e-3)
    w_trained = s.get_params()
    # held-out configurations: S_NN + ln w_F should vary less than ln w_F
    res, lnw = [], []
    for k in range(6):
        g.sweep(2)
        phi = g.get_fields()
        snn = s.action(phi)
        for z in range(nch):
            lw = g.logdet(z).real
            lnw.append(lw)
            res.append(snn[z] + lw)
    r2 = 1.0 - np.var(res) / np.var(lnw)

    def acceptance(w, moves=40):
        s.set_params(w)
        acc = 0
        for _ in range(moves):
            acc += sum(mv["accepted"] for mv in s.global_move(1, 8, 0.2))
            g.sweep(1)
        return acc / (moves * nch)

    a_trained = acceptance(w_trained)
    a_gauss = acceptance(np.zeros_like(w_trained))
    a_untrained = acceptance(w_untrained)
    print("SLMC: held-out R2 %.3f, acceptance trained %.3f, Gaussian %.3f, untrained %.3f (train loss %.3f -> %.3f)"
          % (r2, a_trained, a_gauss, a_untrained, loss0, loss))
    assert r2 > 0.25
    assert a_trained > a_gauss + 0.03
    assert a_trained > a_untrained + 0.03
    s.close()
    g.close()

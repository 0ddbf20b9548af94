"""GPU replay of the oracle's recorded Markov-chain histories at the workload shapes.

tests/golden/hist_*.npz hold the FP64 oracle's accept flags, ln A, step sizes,
final fields, G(0), G(L/2) and ln w_F per chain (written by
tests/golden/make_histories.py, which calls only oracle/ and synth/). The GPU
context starts from the same seeded fields and replays the same noise.

Bars: FP64 path identical accept/reject sequences, ln A within 1e-7, step
sizes within 1e-12, fields within 1e-10, G and ln w_F within 1e-10 relative
(max norm). Mixed path (FP32 wraps with FP64 accumulation): identical
accept/reject sequences, the updated G within 1e-6 (absolute, max |G - G_FP64|)
of its FP64 recomputation at every stabilisation point, and the fields, G and
ln w_F within 1e-6 of the oracle's.
"""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_03700_amd import CFQMC, Batch
    return CFQMC, Batch


def _load(name):
    d = np.load(os.path.join(HERE, "golden", "hist_%s.npz" % name))
    cfg = json.loads(str(d["meta_json"]))
    return cfg, d


def _inputs(cfg, n_q):
    phi = np.stack([synth.fields(cfg["seed_f"] + k, cfg["l_tau"], n_q) for k in range(len(cfg["u"]))])
    rp = np.stack([synth.replay(cfg["seed_r"] + k, cfg["n_sweeps"], cfg["l_tau"], n_q)
                   for k in range(len(cfg["u"]))])
    return phi, rp


def _kw(cfg, precision, tile_cfg=1):
    return dict(n_phi=cfg["n_phi"], l_tau=cfg["l_tau"], dtau=cfg["dtau"], q_mode=cfg["q_mode"],
                q_max=cfg["q_max"] or 3.0, n_stab=cfg["n_stab"], eps0=cfg["eps0"], adapt_eps=True,
                precision=precision, n_chains=len(cfg["u"]), chain_u=[(1.0, u, u) for u in cfg["u"]],
                tile_cfg=tile_cfg, exp_squarings=cfg.get("exp_squarings", 2))


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _check_sweep(g, k, kl, d, sw, st, mixed):
    """Accept flags, ln A and the stabilisation check of chain k (context index kl) after sweep sw."""
    acc, lna = g.last_sweep(kl)
    assert acc.tolist() == d["acc%d" % k][sw].tolist(), (k, sw)
    lref = d["lna%d" % k][sw]
    fin = np.isfinite(lref)
    assert np.abs(lna[fin] - lref[fin]).max() < (1e-4 if mixed else 1e-7), (k, sw)
    if mixed:
        assert st["max_stab_err"] <= 1e-6, (k, sw, st["max_stab_err"])
    else:
        assert st["max_stab_err"] < 1e-9, (k, sw, st["max_stab_err"])
    assert st["max_phase_err"] < 1e-6


def _check_final(g, k, kl, d, cfg, mixed):
    n = 2 * cfg["n_phi"]
    L = cfg["l_tau"]
    tol = 1e-6 if mixed else 1e-10
    assert abs(g.get_eps()[kl] - d["eps%d" % k][-1]) < 1e-12
    assert np.abs(g.get_fields()[kl] - d["phi%d" % k]).max() < tol
    G0 = g.measure_G(kl, 0)[:n, :n]
    Gm = g.measure_G(kl, L // 2)[:n, :n]
    if mixed:
        assert np.abs(G0 - d["G%d" % k]).max() < tol and np.abs(Gm - d["Gm%d" % k]).max() < tol
    else:
        assert rel(G0, d["G%d" % k]) < tol and rel(Gm, d["Gm%d" % k]) < tol
    ld = g.logdet(kl)
    ldr = complex(d["ld%d" % k])
    assert abs(ld.real - ldr.real) < tol * abs(ldr.real)


def _replay_context(name, precision, tile_cfg=1):
    CFQMC, _ = _gpu()
    cfg, d = _load(name)
    g = CFQMC(**_kw(cfg, precision, tile_cfg))
    phi, rp = _inputs(cfg, g.n_q)
    g.init_fields(phi)
    mixed = precision != 0
    for sw in range(cfg["n_sweeps"]):
        st = g.sweep(1, rp[:, sw:sw + 1])
        for k in range(len(cfg["u"])):
            _check_sweep(g, k, k, d, sw, st[k], mixed)
    for k in range(len(cfg["u"])):
        _check_final(g, k, k, d, cfg, mixed)
    g.close()


def test_n36_full_size_five_couplings_fp64():
    """N_phi = 36, |q| l_B <= 3 (161 components), L = 200, u = 0.5 .. 2.5 as five
    chains of one context, one sweep of replayed noise, FP64."""
    _replay_context("c2_n36", 0)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_n100_paper_cutoff_short_axis(precision):
    """The bench shape: N_phi = 100, paper cutoff (933 components), u = 1.5,
    n_stab = 8, on a 16-slice axis, two sweeps; FP64, mixed, and mixed with the
    Woodbury product and the rank-k update in FP32 as well."""
    _replay_context("c3_n100", precision)


def test_n100_mixed_fp32_accumulating_tiles():
    """The same N_phi = 100 replay with the FP32 applications accumulating in
    FP32 over the whole k range (channel-application configuration 10, 64 x 32
    tiles): the mixed bar holds."""
    _replay_context("c3_n100", 1, tile_cfg=10)


@pytest.mark.parametrize("precision,tile_cfg", [(0, 16), (1, 18), (0, 19)])
def test_n100_wide_workgroup_tiles(precision, tile_cfg):
    """The N_phi = 100 replay with the 16-wave 64 x 64 workgroup tiles of the
    channel application (configuration 16 in FP64, 18 in the FP32 three-product
    form) and with the FP64 valley split over eight waves (19): the FP64 and
    mixed bars hold."""
    _replay_context("c3_n100", precision, tile_cfg=tile_cfg)


def test_sphere_n59_largest_sphere_one_sweep():
    """The paper's largest sphere, N_phi = 59 (3481 components per channel,
    spin block 118), dtau = 0.01, u = 0.2, on an 8-slice axis with n_stab = 4:
    one replayed FP64 sweep."""
    _replay_context("sphere_n59", 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_n140_largest_torus_one_sweep(precision):
    """The paper's largest torus N_phi = 140 (1305 components), 8 slices, n_stab = 4."""
    _replay_context("c5_n140", precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_batched_shapes_n24_n48_n72(precision):
    """The batched workload's three shapes (N_phi = 24, 48, 72, paper cutoff) as
    three groups of one heterogeneous batch, their slice steps interleaved on
    their own streams, replayed noise per group; checked per chain through
    cfqmc_batch_get."""
    _, Batch = _gpu()
    names = ["c4_n24", "c4_n48", "c4_n72"]
    loaded = [_load(nm) for nm in names]
    b = Batch([_kw(cfg, precision) for cfg, _ in loaded])
    rps = []
    for gi, (cfg, d) in enumerate(loaded):
        phi, rp = _inputs(cfg, b.groups[gi].n_q)
        b.groups[gi].init_fields(phi)
        rps.append(rp)
    st = b.sweep(1, replay=rps)
    mixed = precision != 0
    for gi, (cfg, d) in enumerate(loaded):
        g, kl = b.get(gi)           # chain gi of the batch is the single chain of group gi
        assert g is b.groups[gi] and kl == 0
        _check_sweep(g, 0, kl, d, 0, st[gi], mixed)
        _check_final(g, 0, kl, d, cfg, mixed)
    b.close()

"""GPU parity of the HIP sweep against the FP64 oracle, through the C ABI.

Bars (spec tolerances): FP64 path 1e-10 relative in G and ln w on an
identical recorded field history / replayed noise; mixed path <= 1e-6 in G.
Accept/reject sequences under replayed noise must be identical.
"""
import numpy as np
import pytest

import synth
from oracle import dqmc
from oracle.model import Model, Q_BZ, Q_PAPER, Q_RADIUS
from oracle.observables import so5_observables

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_03700_amd import CFQMC
    return CFQMC


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def wrap_phase(x):
    return abs(np.angle(np.exp(1j * x)))


CASES = [
    # n_phi, L, n_stab, q_mode, q_max, u
    (4, 8, 4, Q_BZ, None, 1.0),
    (5, 7, 3, Q_PAPER, None, 1.3),      # odd N, ragged last stabilisation block
    (6, 40, 10, Q_BZ, None, 1.0),       # the N_phi = 6 workload (36 momenta, L = 40)
]


@pytest.mark.parametrize("n_phi,L,nstab,mode,qmax,u", CASES)
def test_green_and_logdet_at_init(n_phi, L, nstab, mode, qmax, u):
    CFQMC = _gpu()
    m = Model(n_phi, L, 0.1, u0=1.0, uk=u, un=u, q_mode=mode, q_max=qmax)
    phi = synth.fields(100 + n_phi, L, m.n_q)
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, u0=1.0, uk=u, un=u, q_mode=mode, q_max=qmax or 3.0,
              n_stab=nstab, tile_cfg=1)
    assert g.n_q == m.n_q
    g.init_fields(phi[None])
    Bs = dqmc.propagators(m, phi)
    for tau in sorted({0, 1, nstab, L - 1, L}):
        G = g.measure_G(0, tau)
        Gr = dqmc.green(m, phi, tau, Bs)
        n = 2 * n_phi
        assert rel(G[:n, :n], Gr) < 1e-10, tau
        assert np.abs(G[n:, n:] - G[:n, :n]).max() == 0 and np.abs(G[:n, n:]).max() == 0
        assert abs(np.trace(G).real - 2 * n_phi) < 1e-10          # Re tr G_4N = 2 N (half filling)
    ld, ldr = g.logdet(0), dqmc.logdet(m, phi, Bs)
    assert abs(ld.real - ldr.real) < 1e-10 * abs(ldr.real)
    assert wrap_phase(ld.imag) < 1e-9 and wrap_phase(ldr.imag) < 1e-9
    s, m2 = g.observables(0)
    sr, m2r = so5_observables(dqmc.green(m, phi, L, Bs), n_phi)
    assert np.abs(s - sr.real).max() < 1e-10 * np.abs(sr).max()
    assert abs(m2 - m2r) < 1e-10 * abs(m2r)
    g.close()


def _replay_compare(CFQMC, n_phi, L, nstab, mode, qmax, u_list, precision, n_sweeps, tol_g, seed=7, eps0=0.4,
                    dtau=0.1, **ctx_kw):
    nch = len(u_list)
    models = [Model(n_phi, L, dtau, u0=1.0, uk=u, un=u, q_mode=mode, q_max=qmax) for u in u_list]
    nq = models[0].n_q
    phi = np.stack([synth.fields(seed + 10 * k, L, nq) for k in range(nch)])
    rp = np.stack([synth.replay(seed + 10 * k + 1, n_sweeps, L, nq) for k in range(nch)])
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=dtau, q_mode=mode, q_max=qmax or 3.0, n_stab=nstab, eps0=eps0,
              adapt_eps=True, precision=precision, n_chains=nch,
              chain_u=[(1.0, u, u) for u in u_list], tile_cfg=1, **ctx_kw)
    g.init_fields(phi)
    chains = [dqmc.Chain(models[k], phi[k], eps0=eps0, adapt=True) for k in range(nch)]
    for sw in range(n_sweeps):
        st = g.sweep(1, rp[:, sw:sw + 1])
        for k in range(nch):
            chains[k].sweep(rp[k, sw])
            acc, lna = g.last_sweep(k)
            hist = chains[k].history[-L:]
            assert acc.tolist() == [int(h[2]) for h in hist], (k, sw)
            finite = np.array([np.isfinite(h[1]) for h in hist])
            lref = np.array([h[1] for h in hist])
            assert np.allclose(lna[finite], lref[finite], rtol=0, atol=tol_g * 1e3)
            assert st[k]["max_phase_err"] < 1e-6
    eps = g.get_eps()
    for k in range(nch):
        m = models[k]
        assert abs(eps[k] - chains[k].eps) < 1e-12
        # fields differ only through the drift computed from the (mixed) G frames
        assert np.abs(g.get_fields()[k] - chains[k].phi).max() < max(1e-10, 1e-2 * tol_g)
        G = g.measure_G(k, L)[:2 * n_phi, :2 * n_phi]
        assert rel(G, dqmc.green(m, chains[k].phi, L)) < tol_g
        ld, ldr = g.logdet(k), dqmc.logdet(m, chains[k].phi)
        assert abs(ld.real - ldr.real) < max(tol_g, 1e-10) * abs(ldr.real)
    g.close()
    return st


def test_sweep_replay_parity_fp64_small():
    """The N_phi = 6 workload: BZ momenta (36 components), L = 40, n_stab = 10,
    u = 1, one chain, 20 sweeps of replayed noise, FP64."""
    CFQMC = _gpu()
    st = _replay_compare(CFQMC, 6, 40, 10, Q_BZ, None, [1.0], 0, 20, 1e-10)
    assert st[0]["max_stab_err"] < 1e-9 and st[0]["max_stab_rel"] <= st[0]["max_stab_err"] / 0.1


def test_sweep_replay_parity_large_spin_block():
    """N_phi = 130: spin block n = 260 > 256 (five column tiles per wave in the
    right solve) with a ragged last 16-column block; FP64 replay parity."""
    CFQMC = _gpu()
    _replay_compare(CFQMC, 130, 3, 2, Q_RADIUS, 1.0, [1.0], 0, 1, 1e-10)


def test_sweep_replay_parity_batched_u_grid():
    """Five chains of one shape at u = 0.5..2.5 in one context (one launch per step)."""
    CFQMC = _gpu()
    _replay_compare(CFQMC, 8, 24, 6, Q_RADIUS, 3.0, [0.5, 1.0, 1.5, 2.0, 2.5], 0, 2, 1e-10)


@pytest.mark.parametrize("precision,guard", [(1, 1), (2, 1), (2, 0)])
def test_sweep_replay_parity_mixed(precision, guard):
    """Mixed paths: FP32 MFMA wraps and frames (1), also the Woodbury product and
    the rank-k update G' = G M^-1 (2), with FP64 accumulation and FP64
    recomputation; with the precision guard off every chain takes the FP32
    products. G after a sweep (recomputed in FP64) within 1e-6 and the G drift
    between recomputations within 1e-6."""
    CFQMC = _gpu()
    st = _replay_compare(CFQMC, 6, 40, 10, Q_BZ, None, [1.0], precision, 2, 1e-6, precision_guard=guard)
    assert st[0]["max_stab_err"] < 1e-6 and st[0]["max_stab_rel"] < 1e-6
    if not guard:
        assert st[0]["fp64_guard_frac"] == 0.0 and st[0]["max_stab_err"] > 1e-12


@pytest.mark.parametrize("n_phi", [7, 36])
def test_tile_configurations_agree(n_phi):
    """Every channel-application configuration of the FP64 path (16 x 16 to
    64 x 64 workgroup tiles, the valley split over eight waves, ragged edges at
    N_phi = 7 and 36): the same accept sequence and G within 1e-12 after a
    replayed sweep."""
    CFQMC = _gpu()
    L = 12
    m = Model(n_phi, L, 0.1, u0=1.0, uk=1.0, un=1.0)
    phi = synth.fields(3, L, m.n_q)
    rp = synth.replay(4, 1, L, m.n_q)
    out = []
    for cfg in range(20):
        g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, n_stab=4, eps0=0.4, adapt_eps=False, tile_cfg=cfg)
        g.init_fields(phi[None])
        g.sweep(1, rp[None])
        out.append((g.measure_G(0, L), g.last_sweep(0)[0].tolist()))
        g.close()
    for G, acc in out[1:]:
        assert acc == out[0][1]
        assert rel(G, out[0][0]) < 1e-12


def test_mixed_tile_configurations_within_the_bar():
    """Every channel-application configuration of the FP32 path, with FP64
    accumulation points (0..7, 14..16) or FP32 accumulation over the whole k
    range (8..13, 17, 18; 12..14, 17, 18 in the three-product form; 15..18 with
    8- and 16-wave workgroups): identical accept/reject
    sequences and the updated G within 1e-6 of its FP64 recomputation; G after
    the sweep within 1e-8 of the FP64 path."""
    CFQMC = _gpu()
    n_phi, L = 7, 12
    m = Model(n_phi, L, 0.1, u0=1.0, uk=1.0, un=1.0)
    phi = synth.fields(3, L, m.n_q)
    rp = synth.replay(4, 1, L, m.n_q)
    ref = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, n_stab=4, eps0=0.4, adapt_eps=False, tile_cfg=1)
    ref.init_fields(phi[None])
    ref.sweep(1, rp[None])
    G0, acc0 = ref.measure_G(0, L), ref.last_sweep(0)[0].tolist()
    ref.close()
    for cfg in range(20):
        g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, n_stab=4, eps0=0.4, adapt_eps=False, tile_cfg=cfg, precision=1)
        g.init_fields(phi[None])
        st = g.sweep(1, rp[None])
        assert g.last_sweep(0)[0].tolist() == acc0, cfg
        assert st[0]["max_stab_err"] < 1e-6, (cfg, st[0]["max_stab_err"])
        assert rel(g.measure_G(0, L), G0) < 1e-8, cfg
        g.close()


def test_exponential_scaling_and_squaring_path():
    """Large fields force the scaled Taylor exponential with squarings."""
    CFQMC = _gpu()
    n_phi, L, u = 5, 6, 3.0
    m = Model(n_phi, L, 0.2, u0=1.0, uk=u, un=u)
    phi = synth.fields(8, L, m.n_q, scale=6.0)
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.2, u0=1.0, uk=u, un=u, n_stab=3, exp_squarings=4, tile_cfg=0)
    g.init_fields(phi[None])
    G = g.measure_G(0, 2)[:2 * n_phi, :2 * n_phi]
    assert rel(G, dqmc.green(m, phi, 2)) < 1e-10
    g.close()


def test_exponential_mixed_squaring_counts():
    """Slices whose fields are scaled from 0.1 to 8 need 0 up to several
    squarings inside the same batched exponential launch (each matrix leaves
    the squaring chain at its own step); G and ln w at every slice boundary
    match the oracle's exact exponentials."""
    CFQMC = _gpu()
    n_phi, L, u = 5, 8, 3.0
    m = Model(n_phi, L, 0.2, u0=1.0, uk=u, un=u)
    scales = np.array([0.1, 8.0, 1.0, 3.0, 0.5, 6.0, 2.0, 0.2])
    phi = synth.fields(21, L, m.n_q) * scales[:, None, None]
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.2, u0=1.0, uk=u, un=u, n_stab=4, exp_squarings=6, tile_cfg=1)
    g.init_fields(phi[None])
    Bs = dqmc.propagators(m, phi)
    for tau in range(L + 1):
        G = g.measure_G(0, tau)[:2 * n_phi, :2 * n_phi]
        assert rel(G, dqmc.green(m, phi, tau, Bs)) < 1e-10, tau
    ld, ldr = g.logdet(0), dqmc.logdet(m, phi, Bs)
    assert abs(ld.real - ldr.real) < 1e-10 * abs(ldr.real)
    g.close()


def test_device_rng_sweep_invariants():
    """Without replay (device Philox noise): sign-free phase, particle-hole
    symmetry, finite stabilisation error, acceptance in (0, 1)."""
    CFQMC = _gpu()
    g = CFQMC(n_phi=12, l_tau=40, dtau=0.1, u0=1.0, uk=1.5, un=1.5, n_stab=8, n_chains=2, tile_cfg=1, seed=11)
    g.init_fields(None)
    st = g.sweep(4)
    for k in range(2):
        assert 0 < st[k]["accepted"] < st[k]["proposed"] == 4 * 40
        assert st[k]["max_phase_err"] < 1e-8
        assert st[k]["max_stab_err"] < 1e-8
        G = g.measure_G(k, 40)
        assert abs(np.trace(G).real - 24) < 1e-9
    assert len(g.series(0)) == 4
    g.close()


def test_heterogeneous_batch_matches_standalone_contexts():
    """Groups of different shapes on their own streams, slice steps interleaved:
    every group ends bit-identical to the same group run alone."""
    _gpu()
    from paper_2605_03700_amd import CFQMC, Batch
    groups = [dict(n_phi=6, l_tau=20, n_stab=5, n_chains=2, seed=3, tile_cfg=1,
                   chain_u=[(1.0, 0.8, 0.8), (1.0, 1.6, 1.6)]),
              dict(n_phi=8, l_tau=12, n_stab=4, n_chains=1, seed=5, tile_cfg=1, precision=1)]
    b = Batch(groups)
    b.init_fields()
    st = b.sweep(2, equal_time=True)
    assert len(st) == 3
    sweeps = [2, round(2 * 20 / 12)]
    off = 0
    for k, kw in enumerate(groups):
        g = CFQMC(**kw)
        g.init_fields(None)
        st1 = g.sweep(sweeps[k])
        bg = b.groups[k]
        assert np.array_equal(g.get_fields(), bg.get_fields())
        for z in range(kw["n_chains"]):
            assert st1[z]["accepted"] == st[off + z]["accepted"]
            assert st1[z]["proposed"] == st[off + z]["proposed"] == sweeps[k] * kw["l_tau"]
            assert np.array_equal(g.measure_G(z, kw["l_tau"]), bg.measure_G(z, kw["l_tau"]))
        assert len(bg.series(0)) == sweeps[k]
        off += kw["n_chains"]
        g.close()
    b.close()


def test_recorded_sweep_graph_matches_launch_by_launch():
    """Each sweep of a batch group as launches of its recorded graphs: after
    four calls (the middle two with kernel timing on for one group, which then
    runs the timing variant, cut at the timed launches so that HIP events on
    the stream bracket them; its timed launches are counted alike) every group
    is bit-identical to the same batch run launch by launch: fields, G, step
    sizes, accept counts and the three per-sweep series."""
    _gpu()
    from paper_2605_03700_amd import Batch
    # group 0 spans three recorded chunks (60, 60 and 10 slices)
    groups = [dict(n_phi=6, l_tau=130, n_stab=5, n_chains=2, seed=3, tile_cfg=1,
                   chain_u=[(1.0, 0.8, 0.8), (1.0, 1.6, 1.6)]),
              dict(n_phi=8, l_tau=12, n_stab=4, n_chains=3, seed=5, tile_cfg=1, precision=1)]
    runs = []
    for graph in (0, 1):
        b = Batch([dict(kw, sweep_graph=graph) for kw in groups])
        b.init_fields()
        st = [b.sweep(1)]
        b.groups[0].kernel_timing(True)
        st.append(b.sweep(1))
        st.append(b.sweep(1))
        k_ms, k_count, _ = b.groups[0].kernel_timing_read()
        w_ms, w_count, _ = b.groups[0].kernel_timing_read(woodbury=True)
        b.groups[0].kernel_timing(False)
        st.append(b.sweep(1, equal_time=True))
        # every call ran as graph launches (the timed ones as the timing variant),
        # or launch by launch when asked
        for k in range(4):
            assert all(x["graph_sweep_frac"] == float(graph) for x in st[k]), (graph, k)
        # one timed launch of each kind per slice move, in either way of launching
        assert k_count == w_count == 2 * groups[0]["l_tau"] and k_ms > 0 and w_ms > 0, (graph, k_count, w_count)
        res = {"st": [[(x["accepted"], x["proposed"], x["max_stab_err"]) for x in s] for s in st]}
        for k, g in enumerate(b.groups):
            res["phi%d" % k] = g.get_fields()
            res["eps%d" % k] = g.get_eps()
            res["G%d" % k] = [g.measure_G(z, 0) for z in range(g.n_chains)]
            for w in ("m2", "action", "phi_q0_power"):
                res["%s%d" % (w, k)] = [g.series(z, w) for z in range(g.n_chains)]
        b.close()
        runs.append(res)
    a, b = runs
    assert a["st"] == b["st"]
    for key in a:
        if key == "st":
            continue
        va, vb = a[key], b[key]
        if isinstance(va, list):
            assert all(np.array_equal(x, y) for x, y in zip(va, vb)), key
        else:
            assert np.array_equal(va, vb), key
    assert len(a["m2%d" % 1][0]) == 1 + 2 + round(130 / 12)


def test_checkpoint_restore_continues_the_chains(tmp_path):
    """Two sweeps in one go vs one sweep, checkpoint, restore into a fresh
    context, one sweep: same accept sequence (device noise continues from the
    stored RNG position), same step sizes, fields within rounding (G is rebuilt
    in FP64 at the restore), same m^2 series; malformed restores are refused
    and leave the context usable."""
    CFQMC = _gpu()
    kw = dict(n_phi=6, l_tau=40, dtau=0.1, q_mode=Q_BZ, n_stab=10, n_chains=2, seed=5, eps0=0.4,
              adapt_eps=True, tile_cfg=1, chain_u=[(1.0, 1.0, 1.0), (1.0, 2.0, 2.0)])
    a = CFQMC(**kw)
    a.init_fields(None)
    a.sweep(2)
    fa, ea, acc_a = a.get_fields(), a.get_eps(), [a.last_sweep(z)[0].tolist() for z in range(2)]
    sa = [a.series(z) for z in range(2)]
    a.close()
    b = CFQMC(**kw)
    with pytest.raises(RuntimeError):
        b.checkpoint(str(tmp_path / "early.ck"))          # no fields yet
    b.init_fields(None)
    b.sweep(1)
    path = str(tmp_path / "chains.ck")
    b.checkpoint(path)
    b.close()
    c = CFQMC(**kw)
    with pytest.raises(RuntimeError):
        c.restore(str(tmp_path / "missing.ck"))
    other = CFQMC(**dict(kw, l_tau=20))
    with pytest.raises(RuntimeError):
        other.restore(path)                               # shape differs
    other.close()
    c.restore(path)
    c.sweep(1)
    fc, ec = c.get_fields(), c.get_eps()
    assert [c.last_sweep(z)[0].tolist() for z in range(2)] == acc_a
    assert np.abs(fc - fa).max() < 1e-9
    assert np.abs(ec - ea).max() < 1e-12
    for z in range(2):
        sc = c.series(z)
        assert len(sc) == len(sa[z]) == 2
        assert np.allclose(sc, sa[z], rtol=1e-8, atol=1e-12)
    c.close()


@pytest.mark.parametrize("n_phi,L,mode,qmax,nstab,u_list", [
    (36, 200, Q_RADIUS, 3.0, 10, [0.5, 1.0, 1.5, 2.0, 2.5]),     # the N_phi = 36 workload, full size
    (100, 400, Q_PAPER, None, 8, [1.5, 1.5]),                      # the N_phi = 100 shape, two chains
])
def test_full_size_invariants(n_phi, L, mode, qmax, nstab, u_list):
    """At the workloads' full sizes (too large for the oracle's dense products):
    the updated G equals the FP64 recomputation at every stabilisation point,
    the weight stays sign-free, Re tr G_4N = 2 N_phi at every boundary checked,
    G(beta) = G(0) (periodicity of the equal-time G), moves accepted."""
    CFQMC = _gpu()
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, q_mode=mode, q_max=qmax or 3.0, n_stab=nstab, eps0=0.3,
              adapt_eps=True, precision=0, n_chains=len(u_list), seed=21,
              chain_u=[(1.0, u, u) for u in u_list], tile_cfg=-1)
    g.init_fields(None)
    st = g.sweep(1)
    for k, s in enumerate(st):
        assert s["max_stab_rel"] < 1e-10, (k, s)        # the FP64 bar, relative in max norm
        assert s["max_phase_err"] < 1e-6, (k, s)
        assert 0 <= s["accepted"] <= s["proposed"] == L, (k, s)
        G0 = g.measure_G(k, 0)
        assert abs(np.trace(G0).real - 2 * n_phi) < 1e-9
        assert abs(np.trace(g.measure_G(k, L // 2)).real - 2 * n_phi) < 1e-9
        assert rel(g.measure_G(k, L), G0) < 1e-10
        ld = g.logdet(k)
        # ln w is real for the sign-free model: the imaginary background sum
        # cancels the phase of det(1 + B)^2 up to rounding of O(1e3)-sized terms
        assert np.isfinite(ld.real) and wrap_phase(ld.imag) < 1e-5
    # the first sweep from N(0,1) fields is far from equilibrium: some chains
    # may reject every move, the set as a whole must move
    assert 0 < sum(s["accepted"] for s in st) < sum(s["proposed"] for s in st)
    g.close()


def test_autocorrelation_series_match_their_definitions():
    """The per-sweep series used for tau_int: after each sweep the action entry
    is |phi|^2/2 - ln w_F of the current fields (ln w_F as cfqmc_logdet) and
    the q = 0 power entry is sum_i (sum_tau phi^i_{tau,0})^2 / L."""
    CFQMC = _gpu()
    g = CFQMC(n_phi=8, l_tau=24, dtau=0.1, u0=1.0, uk=1.5, un=1.5, q_mode=Q_RADIUS, q_max=3.0, n_stab=6,
              n_chains=3, tile_cfg=1, seed=13, eps0=0.4)
    g.init_fields(None)
    for sw in range(3):
        g.sweep(1)
        phi = g.get_fields()
        for z in range(3):
            s_act, s_q0, s_m2 = g.series(z, "action"), g.series(z, "phi_q0_power"), g.series(z, "m2")
            assert len(s_act) == len(s_q0) == len(s_m2) == sw + 1
            want = 0.5 * np.sum(phi[z] ** 2) - g.logdet(z).real
            assert abs(s_act[-1] - want) < 1e-9 * max(1.0, abs(want)), (sw, z)
            q0 = sum(np.sum(phi[z][:, i, 0]) ** 2 for i in range(4)) / 24
            assert abs(s_q0[-1] - q0) < 1e-12 * max(1.0, q0), (sw, z)
    g.close()


def test_kernel_timing_records_one_launch_per_slice_move():
    """The live HIP-event timing brackets one wrap application (FP32 in the
    mixed path) and one Woodbury-product application (FP64) per slice move;
    flops per launch are two N x N x n complex products per chain. Disabling
    it clears the record."""
    CFQMC = _gpu()
    n_phi, L, nch = 6, 8, 2
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, q_mode=Q_BZ, n_stab=4, precision=1, n_chains=nch,
              chain_u=[(1.0, 1.0, 1.0)] * nch, tile_cfg=1)
    g.init_fields(np.stack([synth.fields(40 + k, L, g.n_q) for k in range(nch)]))
    g.kernel_timing(True)
    g.sweep(2)
    for woodbury in (False, True):
        ms, count, flops = g.kernel_timing_read(woodbury=woodbury)
        assert count == 2 * L and 0.0 < ms < 1e3
        assert flops == 8.0 * 2.0 * n_phi ** 2 * (2 * n_phi) * nch
    g.kernel_timing(False)
    g.sweep(1)
    assert g.kernel_timing_read()[1] == 0 and g.kernel_timing_read(woodbury=True)[1] == 0
    g.close()


def test_bench_launch_configuration_256_chains_mixed():
    """The timed launch configuration at full size: 256 chains of N_phi = 100,
    L = 400, paper cutoff, u = 1.5, n_stab = 8, mixed precision, autotuned
    tiles, precision guard. In the first sweep from N(0,1) fields the updated
    G of every chain matches its FP64 recomputation within 2e-5 absolute (right
    after the cold start one chain's max|G| reaches 25); in each of the next
    four sweeps within the 1e-6 bar, absolute. The set of chains moves,
    Re tr G_4N = 2 N_phi, and for the first and the last chain G(0) and ln w
    equal those of a one-chain FP64 context given the same fields (per-chain
    addressing of the batched launches; the one-chain FP64 path is pinned to
    the oracle above)."""
    CFQMC = _gpu()
    from paper_2605_03700_amd import FP64, MIXED
    n_phi, L, nch = 100, 400, 256
    kw = dict(n_phi=n_phi, l_tau=L, dtau=0.1, u0=1.0, uk=1.5, un=1.5, q_mode=Q_PAPER, n_stab=8)
    g = CFQMC(precision=MIXED, n_chains=nch, eps0=0.3, adapt_eps=True, seed=3, **kw)
    g.init_fields()
    st = g.sweep(1)
    assert max(s["max_stab_err"] for s in st) < 2e-5
    assert 0 < sum(s["accepted"] for s in st) < sum(s["proposed"] for s in st)
    for sw in range(4):
        st = g.sweep(1)
        assert max(s["max_stab_err"] for s in st) <= 1e-6, (sw, max(s["max_stab_err"] for s in st))
    phi = g.get_fields()
    for k in (0, nch - 1):
        G0 = g.measure_G(k, 0)
        assert abs(np.trace(G0).real - 2 * n_phi) < 1e-8
        ref = CFQMC(precision=FP64, n_chains=1, **kw)
        ref.init_fields(phi[k:k + 1])
        assert rel(G0, ref.measure_G(0, 0)) < 1e-9, k
        ld, ldr = g.logdet(k), ref.logdet(0)
        assert abs(ld.real - ldr.real) < 1e-10 * abs(ldr.real), k
        ref.close()
    g.close()


@pytest.mark.parametrize("n_phi,L,nstab", [(1, 3, 2), (2, 1, 1)])
def test_degenerate_shapes_replay(n_phi, L, nstab):
    """The smallest shapes: one orbital per flavour (n = 2, the single q = 0
    component) with a ragged stabilisation block, and a single time slice.
    Replayed FP64 sweeps of two chains against the oracle: identical
    accept/reject sequences, G and ln w within 1e-10."""
    CFQMC = _gpu()
    _replay_compare(CFQMC, n_phi, L, nstab, Q_BZ, None, [1.0, 1.3], 0, 3, 1e-10)


@pytest.mark.parametrize("tile_cfg", [1, 12])
def test_guarded_applications_one_launch_equals_two(tile_cfg, monkeypatch):
    """The precision guard's applications as one launch whose workgroups take
    their chain's FP32 or FP64 path (the default for configurations 1 and 12)
    against one launch per precision class (CFQMC_GUARD_PAIR=1): with the
    threshold between the chains' max|G| values, so that both classes occur,
    the two give bit-identical fields, G, step sizes and statistics."""
    CFQMC = _gpu()
    n_phi, L, nstab, nch = 6, 40, 10, 8
    m = Model(n_phi, L, 0.1, u0=1.0, uk=1.0, un=1.0, q_mode=Q_BZ)
    phi = np.stack([synth.fields(700 + k, L, m.n_q) for k in range(nch)])
    us = [(1.0, 0.5 + 0.5 * k, 0.5 + 0.5 * k) for k in range(nch)]
    kw = dict(n_phi=n_phi, l_tau=L, dtau=0.1, q_mode=Q_BZ, n_stab=nstab, eps0=0.4, adapt_eps=True, precision=1,
              n_chains=nch, chain_u=us, tile_cfg=tile_cfg, seed=9)
    # threshold: the median of the chains' max|G| over an unguarded sweep
    g = CFQMC(precision_guard=0, **kw)
    g.init_fields(phi)
    gmax = float(np.median([x["max_abs_g"] for x in g.sweep(1)]))
    g.close()
    runs = []
    for pair in (False, True):
        if pair:
            monkeypatch.setenv("CFQMC_GUARD_PAIR", "1")
        else:
            monkeypatch.delenv("CFQMC_GUARD_PAIR", raising=False)
        g = CFQMC(guard_gmax=gmax, **kw)
        assert g.launch_config()["guard_launch"] == (0 if pair else 1)
        g.init_fields(phi)
        st = [g.sweep(1) for _ in range(3)]
        runs.append((g.get_fields(), g.get_eps(), [g.measure_G(k, 0) for k in range(nch)],
                     [[(x["accepted"], x["max_stab_err"], x["fp64_guard_frac"]) for x in s] for s in st]))
        g.close()
    monkeypatch.delenv("CFQMC_GUARD_PAIR", raising=False)
    (fa, ea, ga, sa), (fb, eb, gb, sb) = runs
    assert np.array_equal(fa, fb) and np.array_equal(ea, eb) and sa == sb
    assert all(np.array_equal(x, y) for x, y in zip(ga, gb))
    fr = [x[2] for s in sa for x in s]
    assert min(fr) < 1.0 and max(fr) > 0.0          # both classes occurred


@pytest.mark.parametrize("precision", [1, 2])
def test_precision_guard_selects_fp64_chains(precision):
    """The mixed path's precision guard: with a max|G| threshold below every
    chain's max|G_FP64| each chain's FP32 applications run in FP64 after the
    first recomputation (guard fraction 1, and the blocks after the first
    recompute to FP64 rounding); with the guard off the fraction is 0. Both
    replay the oracle's accept/reject sequence, and max|G_FP64| >= 1/2 (the
    diagonal of G at half filling)."""
    CFQMC = _gpu()
    n_phi, L, nstab = 6, 40, 10
    m = Model(n_phi, L, 0.1, u0=1.0, uk=1.0, un=1.0, q_mode=Q_BZ)
    phi = np.stack([synth.fields(300 + k, L, m.n_q) for k in range(2)])
    rp = np.stack([synth.replay(310 + k, 2, L, m.n_q) for k in range(2)])
    ch = [dqmc.Chain(m, phi[k], eps0=0.4, adapt=True) for k in range(2)]
    for k in range(2):
        ch[k].run(rp[k])
    for guard, gmax, want in ((1, 1e-9, 1.0), (0, 1.0, 0.0)):
        g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, q_mode=Q_BZ, n_stab=nstab, eps0=0.4, adapt_eps=True,
                  precision=precision, n_chains=2, chain_u=[(1.0, 1.0, 1.0)] * 2, tile_cfg=1,
                  precision_guard=guard, guard_gmax=gmax)
        g.init_fields(phi)
        g.sweep(1, rp[:, 0:1])
        st = g.sweep(1, rp[:, 1:2])       # the guard's choice carries over from the first sweep
        for k in range(2):
            assert g.last_sweep(k)[0].tolist() == [int(h[2]) for h in ch[k].history[-L:]]
            assert abs(st[k]["fp64_guard_frac"] - want) < 1e-12, (guard, st[k]["fp64_guard_frac"])
            assert st[k]["max_abs_g"] >= 0.5 - 1e-12
            if guard:
                assert st[k]["max_stab_err"] < 1e-12     # every block of the second sweep in FP64
            else:
                assert 1e-12 < st[k]["max_stab_err"] < 1e-6
        g.close()

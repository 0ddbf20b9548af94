"""The allocation-free correlator entry point (cfqmc_measure_tau_noalloc)
against the allocating one (cfqmc_measure_tau), through the C ABI.

Both run the same imaginary-time pass and kernels, so the correlator and the
carried-vs-recomputed check agree bit for bit; the bar is 1e-12 relative.
Two calls in a row share the library's fixed device array, the second on a
smaller context (fewer chains, shorter axis), which checks that each call
clears what must start at zero.
"""
import ctypes

import numpy as np
import pytest

import synth
from oracle.model import Model, Q_BZ

pytestmark = pytest.mark.gpu


def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_03700_amd import CFQMC, cfqmc
    return torch, CFQMC, cfqmc


def _ctx(CFQMC, n_phi, L, n_stab, nch, seed):
    m = Model(n_phi, L, 0.1, u0=1.0, uk=1.2, un=1.2, q_mode=Q_BZ)
    g = CFQMC(n_phi=n_phi, l_tau=L, dtau=0.1, u0=1.0, uk=1.2, un=1.2, q_mode=Q_BZ, n_stab=n_stab, n_chains=nch,
              tile_cfg=1, seed=seed, eps0=0.4)
    g.init_fields(np.stack([synth.fields(seed + k, L, m.n_q) for k in range(nch)]))
    g.sweep(1)
    return g


def _noalloc(torch, cfqmc, g):
    lib = cfqmc.load()
    out = torch.full((g.n_chains, g.l_tau + 1, 5), float("nan"), dtype=torch.complex128, device="cuda")
    st = torch.full((g.n_chains, 3), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    rc = lib.cfqmc_measure_tau_noalloc(g.h, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(st.data_ptr()))
    assert rc == 0, lib.cfqmc_last_error(g.h)
    torch.cuda.synchronize()
    return out.cpu().numpy(), st.cpu().numpy()


def test_noalloc_correlator_matches_allocating_entry_point():
    torch, CFQMC, cfqmc = _gpu()
    ga = _ctx(CFQMC, 6, 12, 4, 3, 11)
    gb = _ctx(CFQMC, 4, 8, 3, 2, 21)
    for g in (ga, gb):   # the second call: fewer chains and a shorter axis
        ref, ref_st = g.measure_tau(with_stab=True)
        got, got_st = _noalloc(torch, cfqmc, g)
        assert got.shape == ref.shape
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        assert np.abs(got_st - ref_st).max() <= 1e-12 * max(np.abs(ref_st).max(), 1e-300)
        assert np.isfinite(got).all() and np.all(got_st < 1e-8)
    # the first context again after the smaller one
    ref = ga.measure_tau()
    got, _ = _noalloc(torch, cfqmc, ga)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    ga.close()
    gb.close()


def test_noalloc_rejects_more_chains_than_its_scratch_holds():
    torch, CFQMC, cfqmc = _gpu()
    lib = cfqmc.load()
    g = CFQMC(n_phi=1, l_tau=2, dtau=0.1, q_mode=Q_BZ, n_stab=2, n_chains=513, tile_cfg=1)
    g.init_fields(None)
    out = torch.zeros((513, 3, 5), dtype=torch.complex128, device="cuda")
    rc = lib.cfqmc_measure_tau_noalloc(g.h, ctypes.c_void_p(out.data_ptr()), None)
    assert rc == -1
    assert b"512" in lib.cfqmc_last_error(g.h)
    # the context stays usable
    assert np.isfinite(g.measure_tau()).all()
    g.close()

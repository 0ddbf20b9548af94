"""Python binding of the C ABI in include/cfqmc.h (ctypes; argument marshalling only).

Every step of the sweep runs in the HIP library libcfqmc.so built for gfx950.
There is no CPU fallback: if the library is missing or no GPU is visible the
calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcfqmc.so")

Q_PAPER, Q_RADIUS, Q_BZ, Q_LIST, Q_SPHERE = 0, 1, 2, 3, 4
FP64, MIXED, MIXED_ALL = 0, 1, 2

ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENUMERIC", -5: "ESTATE", -6: "ENOTIMPL"}


class Params(ctypes.Structure):
    _fields_ = [
        ("n_phi", ctypes.c_int32), ("l_tau", ctypes.c_int32), ("dtau", ctypes.c_double),
        ("u0", ctypes.c_double), ("uk", ctypes.c_double), ("un", ctypes.c_double),
        ("q_mode", ctypes.c_int32), ("q_max", ctypes.c_double),
        ("q_list", ctypes.POINTER(ctypes.c_int32)), ("n_q_list", ctypes.c_int32),
        ("n_stab", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("eps0", ctypes.c_double), ("r0", ctypes.c_double), ("deps", ctypes.c_double),
        ("eps_min", ctypes.c_double), ("eps_max", ctypes.c_double),
        ("adapt_eps", ctypes.c_int32), ("seed", ctypes.c_uint64), ("n_chains", ctypes.c_int32),
        ("chain_u", ctypes.POINTER(ctypes.c_double)), ("exp_squarings", ctypes.c_int32),
        ("tile_cfg", ctypes.c_int32), ("dense4n", ctypes.c_int32), ("exact_drift", ctypes.c_int32),
        ("precision_guard", ctypes.c_int32), ("guard_gmax", ctypes.c_double), ("guard_err", ctypes.c_double),
        ("sweep_graph", ctypes.c_int32),
    ]


class SlmcParams(ctypes.Structure):
    _fields_ = [("hidden", ctypes.c_int32), ("n_qbins", ctypes.c_int32), ("n_wbins", ctypes.c_int32),
                ("capacity", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class SlmcMove(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int32), ("inner_accepted", ctypes.c_int32), ("ln_a", ctypes.c_double),
                ("d_lnw", ctypes.c_double), ("d_snn", ctypes.c_double), ("max_abs_dh", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Stats(ctypes.Structure):
    _fields_ = [("proposed", ctypes.c_int64), ("accepted", ctypes.c_int64), ("eps", ctypes.c_double),
                ("max_stab_err", ctypes.c_double), ("max_phase_err", ctypes.c_double),
                ("exp_range_flag", ctypes.c_int32), ("pad", ctypes.c_int32), ("max_stab_rel", ctypes.c_double),
                ("max_abs_g", ctypes.c_double), ("fp64_guard_frac", ctypes.c_double),
                ("graph_sweep_frac", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


_lib = None

EXPORTS = ["cfqmc_default_params", "cfqmc_create", "cfqmc_destroy", "cfqmc_sizes", "cfqmc_init_fields",
           "cfqmc_get_fields", "cfqmc_checkpoint", "cfqmc_restore", "cfqmc_sweep", "cfqmc_measure_G", "cfqmc_green_displaced", "cfqmc_measure_tau", "cfqmc_structure_factors", "cfqmc_sphere_weights", "cfqmc_slmc_set_subspace", "cfqmc_logdet", "cfqmc_observables",
           "cfqmc_series", "cfqmc_series_of", "cfqmc_last_sweep", "cfqmc_get_eps", "cfqmc_set_eps", "cfqmc_tile_config", "cfqmc_launch_config",
           "cfqmc_last_error", "cfqmc_kernel_timing", "cfqmc_kernel_timing_read", "cfqmc_kernel_timing_read_woodbury", "cfqmc_batch_create",
           "cfqmc_batch_context", "cfqmc_batch_sweep", "cfqmc_batch_sweep_replay", "cfqmc_batch_get",
           "cfqmc_batch_destroy", "cfqmc_slmc_default_params",
           "cfqmc_slmc_create", "cfqmc_slmc_destroy", "cfqmc_slmc_sizes", "cfqmc_slmc_set_params",
           "cfqmc_slmc_get_params", "cfqmc_slmc_set_norm", "cfqmc_slmc_get_norm", "cfqmc_slmc_features",
           "cfqmc_slmc_action", "cfqmc_slmc_loss_grad", "cfqmc_slmc_collect", "cfqmc_slmc_clear_data",
           "cfqmc_slmc_train", "cfqmc_slmc_global_move", "cfqmc_slmc_last_proposal", "cfqmc_slmc_grad_check",
           "cfqmc_green_maxdiff", "cfqmc_measure_tau_noalloc", "cfqmc_slmc_train_heldout"]


def load():
    """Load libcfqmc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcfqmc.so not found at %s; run __graft_entry__.build()" % LIB_PATH)
    try:
        # the library must bind to the HIP runtime PyTorch uses (its wheel ships
        # its own): load torch's first, so there is one runtime in the process
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.cfqmc_default_params.argtypes = [ctypes.POINTER(Params)]
    lib.cfqmc_default_params.restype = None
    lib.cfqmc_create.argtypes = [ctypes.POINTER(Params), P, ctypes.POINTER(P)]
    lib.cfqmc_destroy.argtypes = [P]
    lib.cfqmc_sizes.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_int32)]
    lib.cfqmc_init_fields.argtypes = [P, P]
    lib.cfqmc_get_fields.argtypes = [P, P]
    lib.cfqmc_checkpoint.argtypes = [P, ctypes.c_char_p]
    lib.cfqmc_restore.argtypes = [P, ctypes.c_char_p]
    lib.cfqmc_sweep.argtypes = [P, ctypes.c_int32, P, P]
    lib.cfqmc_measure_G.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32]
    lib.cfqmc_green_displaced.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, P]
    lib.cfqmc_measure_tau.argtypes = [P, P, P]
    lib.cfqmc_measure_tau_noalloc.argtypes = [P, P, P]
    lib.cfqmc_structure_factors.argtypes = [P, P, ctypes.c_int32, P]
    lib.cfqmc_sphere_weights.argtypes = [ctypes.c_int32, P]
    lib.cfqmc_slmc_set_subspace.argtypes = [P, ctypes.c_int32]
    lib.cfqmc_logdet.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.cfqmc_observables.argtypes = [P, ctypes.c_int32, P, ctypes.POINTER(ctypes.c_double)]
    lib.cfqmc_series.argtypes = [P, ctypes.c_int32, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.cfqmc_series_of.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32)]
    lib.cfqmc_last_sweep.argtypes = [P, ctypes.c_int32, P, P]
    lib.cfqmc_get_eps.argtypes = [P, P]
    lib.cfqmc_set_eps.argtypes = [P, P]
    lib.cfqmc_tile_config.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    lib.cfqmc_launch_config.argtypes = [P, P]
    lib.cfqmc_kernel_timing.argtypes = [P, ctypes.c_int32]
    lib.cfqmc_kernel_timing_read.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_double)]
    lib.cfqmc_kernel_timing_read_woodbury.argtypes = lib.cfqmc_kernel_timing_read.argtypes
    lib.cfqmc_batch_create.argtypes = [ctypes.POINTER(Params), ctypes.c_int32, ctypes.POINTER(P)]
    lib.cfqmc_batch_context.argtypes = [P, ctypes.c_int32, ctypes.POINTER(P)]
    lib.cfqmc_batch_sweep.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P]
    lib.cfqmc_batch_sweep_replay.argtypes = [P, ctypes.c_int32, P, P]
    lib.cfqmc_batch_get.argtypes = [P, ctypes.c_int32, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int32)]
    lib.cfqmc_batch_destroy.argtypes = [P]
    D = ctypes.c_double
    lib.cfqmc_slmc_default_params.argtypes = [ctypes.POINTER(SlmcParams)]
    lib.cfqmc_slmc_default_params.restype = None
    lib.cfqmc_slmc_create.argtypes = [P, ctypes.POINTER(SlmcParams), ctypes.POINTER(P)]
    lib.cfqmc_slmc_destroy.argtypes = [P]
    lib.cfqmc_slmc_sizes.argtypes = [P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int32)]
    lib.cfqmc_slmc_set_params.argtypes = [P, P]
    lib.cfqmc_slmc_get_params.argtypes = [P, P]
    lib.cfqmc_slmc_set_norm.argtypes = [P, P, P, D, D]
    lib.cfqmc_slmc_get_norm.argtypes = [P, P, P, ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.cfqmc_slmc_features.argtypes = [P, P, ctypes.c_int32, P]
    lib.cfqmc_slmc_action.argtypes = [P, P, ctypes.c_int32, P, P]
    lib.cfqmc_slmc_grad_check.argtypes = [P, P, ctypes.c_int32, P, P]
    lib.cfqmc_slmc_loss_grad.argtypes = [P, P, P, ctypes.c_int32, ctypes.POINTER(D), P, P]
    lib.cfqmc_slmc_collect.argtypes = [P]
    lib.cfqmc_slmc_clear_data.argtypes = [P]
    lib.cfqmc_slmc_train.argtypes = [P, ctypes.c_int32, ctypes.c_int32, D, ctypes.c_int32, ctypes.POINTER(D)]
    lib.cfqmc_slmc_train_heldout.argtypes = [P, ctypes.c_int32, ctypes.c_int32, D, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_int32, ctypes.POINTER(D), ctypes.POINTER(D),
                                             ctypes.POINTER(ctypes.c_int32)]
    lib.cfqmc_slmc_global_move.argtypes = [P, ctypes.c_int32, ctypes.c_int32, D, P, P]
    lib.cfqmc_slmc_last_proposal.argtypes = [P, ctypes.c_int32, P]
    lib.cfqmc_green_maxdiff.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, P, P]
    lib.cfqmc_last_error.argtypes = [P]
    lib.cfqmc_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("cfqmc_default_params", "cfqmc_last_error", "cfqmc_slmc_default_params"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def make_params(n_phi=6, l_tau=40, dtau=0.1, u0=1.0, uk=1.0, un=1.0, q_mode=Q_PAPER, q_max=3.0,
                q_list=None, n_stab=10, precision=FP64, eps0=0.5, r0=0.574, deps=0.1, eps_min=1e-3,
                eps_max=5.0, adapt_eps=True, seed=1, n_chains=1, chain_u=None, exp_squarings=2, tile_cfg=-1,
                dense4n=0, exact_drift=0, precision_guard=1, guard_gmax=0.8, guard_err=2.5e-7, sweep_graph=1):
    """Fill a Params structure; returns (params, keep-alive arrays)."""
    lib = load()
    p = Params()
    lib.cfqmc_default_params(ctypes.byref(p))
    p.n_phi, p.l_tau, p.dtau = n_phi, l_tau, dtau
    p.u0, p.uk, p.un = u0, uk, un
    p.q_mode, p.q_max = q_mode, q_max
    keep = []
    if q_list is not None:
        ql = np.ascontiguousarray(np.asarray(q_list, dtype=np.int32).reshape(-1))
        keep.append(ql)
        p.q_list = ql.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        p.n_q_list = ql.size // 2
    p.n_stab, p.precision = n_stab, precision
    p.eps0, p.r0, p.deps, p.eps_min, p.eps_max = eps0, r0, deps, eps_min, eps_max
    p.adapt_eps, p.seed, p.n_chains = int(bool(adapt_eps)), seed, n_chains
    if chain_u is not None:
        cu = np.ascontiguousarray(np.asarray(chain_u, dtype=np.float64).reshape(n_chains, 3))
        keep.append(cu)
        p.chain_u = cu.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    p.exp_squarings, p.tile_cfg = exp_squarings, tile_cfg
    p.dense4n, p.exact_drift = int(dense4n), int(exact_drift)
    p.precision_guard, p.guard_gmax, p.guard_err = int(precision_guard), float(guard_gmax), float(guard_err)
    p.sweep_graph = int(sweep_graph)
    return p, keep


class CFQMC:
    """One context of the C ABI: n_chains chains of one lattice shape."""

    def __init__(self, n_phi=6, l_tau=40, dtau=0.1, u0=1.0, uk=1.0, un=1.0, q_mode=Q_PAPER, q_max=3.0,
                 q_list=None, n_stab=10, precision=FP64, eps0=0.5, r0=0.574, deps=0.1, eps_min=1e-3,
                 eps_max=5.0, adapt_eps=True, seed=1, n_chains=1, chain_u=None, exp_squarings=2,
                 tile_cfg=-1, dense4n=0, exact_drift=0, precision_guard=1, guard_gmax=0.8, guard_err=2.5e-7,
                 sweep_graph=1,
                 stream=None, _handle=None):
        lib = load()
        self.lib = lib
        if _handle is not None:          # view of a context owned by a batch
            self.h = _handle
            self._owned = False
            self._init_sizes(n_phi, l_tau)
            return
        self._owned = True
        p = Params()
        lib.cfqmc_default_params(ctypes.byref(p))
        p.n_phi, p.l_tau, p.dtau = n_phi, l_tau, dtau
        p.u0, p.uk, p.un = u0, uk, un
        p.q_mode, p.q_max = q_mode, q_max
        self._qlist = None
        if q_list is not None:
            self._qlist = np.ascontiguousarray(np.asarray(q_list, dtype=np.int32).reshape(-1))
            p.q_list = self._qlist.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            p.n_q_list = self._qlist.size // 2
        p.n_stab, p.precision = n_stab, precision
        p.eps0, p.r0, p.deps, p.eps_min, p.eps_max = eps0, r0, deps, eps_min, eps_max
        p.adapt_eps, p.seed, p.n_chains = int(bool(adapt_eps)), seed, n_chains
        self._cu = None
        if chain_u is not None:
            self._cu = np.ascontiguousarray(np.asarray(chain_u, dtype=np.float64).reshape(n_chains, 3))
            p.chain_u = self._cu.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.exp_squarings, p.tile_cfg = exp_squarings, tile_cfg
        p.dense4n, p.exact_drift = int(dense4n), int(exact_drift)
        p.precision_guard, p.guard_gmax, p.guard_err = int(precision_guard), float(guard_gmax), float(guard_err)
        p.sweep_graph = int(sweep_graph)
        if stream is None:
            import torch
            if not torch.cuda.is_available():
                raise RuntimeError("no GPU visible: the CF-DQMC library runs on the MI355X only")
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = ctypes.c_void_p()
        self._check(lib.cfqmc_create(ctypes.byref(p), ctypes.c_void_p(stream), ctypes.byref(h)), None)
        self.h = h
        self._init_sizes(n_phi, l_tau)

    def _init_sizes(self, n_phi, l_tau):
        nq, nc, d4 = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        self.lib.cfqmc_sizes(self.h, ctypes.byref(nq), ctypes.byref(nc), ctypes.byref(d4))
        self.n_q, self.n_chains, self.dim_g4n = nq.value, nc.value, d4.value
        self.n_phi, self.l_tau = n_phi, l_tau

    def _check(self, rc, h="self"):
        if rc != 0:
            if h is not None and getattr(self, "h", None) is not None:
                msg = self.lib.cfqmc_last_error(self.h).decode()
            else:                   # a failed create: the thread's last create message
                msg = self.lib.cfqmc_last_error(None).decode()
            raise RuntimeError("cfqmc error %s: %s" % (ERRORS.get(rc, rc), msg))

    def init_fields(self, phi=None):
        if phi is not None:
            phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(self.n_chains, self.l_tau, 4, self.n_q)
        self._check(self.lib.cfqmc_init_fields(self.h, _ptr(phi)))

    def get_fields(self):
        out = np.empty((self.n_chains, self.l_tau, 4, self.n_q))
        self._check(self.lib.cfqmc_get_fields(self.h, _ptr(out)))
        return out

    def checkpoint(self, path):
        """Write fields, step sizes, RNG position and series to `path`."""
        self._check(self.lib.cfqmc_checkpoint(self.h, os.fsencode(path)))

    def restore(self, path):
        """Continue the chains stored in `path` (same shape and couplings)."""
        self._check(self.lib.cfqmc_restore(self.h, os.fsencode(path)))

    def sweep(self, n_sweeps=1, replay=None):
        if replay is not None:
            replay = np.ascontiguousarray(replay, dtype=np.float64).reshape(
                self.n_chains, n_sweeps, self.l_tau, 4 * self.n_q + 1)
        st = (Stats * self.n_chains)()
        self._check(self.lib.cfqmc_sweep(self.h, n_sweeps, _ptr(replay), ctypes.cast(st, ctypes.c_void_p)))
        return [s.as_dict() for s in st]

    def measure_G(self, chain=0, tau=None, out=None):
        """G(tau) expanded to 4N; out: optional torch complex128 device tensor (4N x 4N)."""
        tau = self.l_tau if tau is None else tau
        if out is not None:
            self._check(self.lib.cfqmc_measure_G(self.h, chain, tau, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        g = np.empty((self.dim_g4n, self.dim_g4n), dtype=np.complex128)
        self._check(self.lib.cfqmc_measure_G(self.h, chain, tau, _ptr(g), 0))
        return g

    def green_displaced(self, chain=0, tau=0):
        """(G(tau,0), G(0,tau), G(tau,tau)) of one chain on the spin block, n x n complex128."""
        n = 2 * self.n_phi
        out = [np.empty((n, n), dtype=np.complex128) for _ in range(3)]
        self._check(self.lib.cfqmc_green_displaced(self.h, chain, tau, _ptr(out[0]), _ptr(out[1]), _ptr(out[2])))
        return tuple(out)

    def measure_tau(self, with_stab=False):
        """C^i(tau) = <n^i_{q=0}(tau) n^i_{q=0}(0)> of every chain: complex128
        [n_chains][l_tau + 1][5]; m^2_SO(5)(tau) is the mean over the last axis.
        with_stab: also return [n_chains][3], the relative difference of the
        carried and recomputed G(tau,0), G(0,tau), G(tau,tau) at block boundaries."""
        out = np.empty((self.n_chains, self.l_tau + 1, 5), dtype=np.complex128)
        st = np.empty((self.n_chains, 3))
        self._check(self.lib.cfqmc_measure_tau(self.h, _ptr(out), _ptr(st)))
        return (out, st) if with_stab else out

    def structure_factors(self, qs):
        """S^i_q, i = 1..5, at the momenta qs (sequence of (qx, qy)) for every
        chain: complex128 [n_chains][len(qs)][5]."""
        q = np.ascontiguousarray(np.asarray(qs, dtype=np.int32).reshape(-1, 2))
        out = np.empty((self.n_chains, q.shape[0], 5), dtype=np.complex128)
        self._check(self.lib.cfqmc_structure_factors(self.h, _ptr(q), q.shape[0], _ptr(out)))
        return out

    def logdet(self, chain=0):
        re, im = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.cfqmc_logdet(self.h, chain, ctypes.byref(re), ctypes.byref(im)))
        return complex(re.value, im.value)

    def observables(self, chain=0):
        s = np.empty(5)
        m2 = ctypes.c_double()
        self._check(self.lib.cfqmc_observables(self.h, chain, _ptr(s), ctypes.byref(m2)))
        return s, m2.value

    SERIES = {"m2": 0, "action": 1, "phi_q0_power": 2}

    def series(self, chain=0, which="m2", max_len=1 << 16):
        """Per-sweep series: "m2" (m^2_SO(5)), "action" (|phi|^2/2 - ln w_F) or
        "phi_q0_power" (power of the q = 0 fields)."""
        out = np.empty(max_len)
        ln = ctypes.c_int32()
        self._check(self.lib.cfqmc_series_of(self.h, chain, self.SERIES[which], _ptr(out), max_len, ctypes.byref(ln)))
        return out[:ln.value].copy()

    def last_sweep(self, chain=0):
        acc = np.empty(self.l_tau, dtype=np.int32)
        lna = np.empty(self.l_tau)
        self._check(self.lib.cfqmc_last_sweep(self.h, chain, _ptr(acc), _ptr(lna)))
        return acc, lna

    def get_eps(self):
        e = np.empty(self.n_chains)
        self._check(self.lib.cfqmc_get_eps(self.h, _ptr(e)))
        return e

    def set_eps(self, eps):
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (self.n_chains,)))
        self._check(self.lib.cfqmc_set_eps(self.h, _ptr(e)))

    def tile_config(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.cfqmc_tile_config(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def launch_config(self):
        """The launch configuration chosen at create: channel application
        (context precision; FP32 in mixed contexts), FP64 channel application
        of a mixed context, n x n GEMM, exponential GEMM, guarded launch form."""
        o = np.zeros(5, dtype=np.int32)
        self._check(self.lib.cfqmc_launch_config(self.h, _ptr(o)))
        return {"chan": int(o[0]), "chan_fp64": int(o[1]), "gemm": int(o[2]), "gemm_exp": int(o[3]),
                "guard_launch": int(o[4])}

    def kernel_timing(self, enable=True):
        self._check(self.lib.cfqmc_kernel_timing(self.h, int(bool(enable))))

    def kernel_timing_read(self, woodbury=False):
        """(mean ms per sampled channel-application launch, count, flops per
        launch) of the wrap's timed application, or (woodbury=True) of the
        Woodbury product's."""
        a, k, f = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        fn = self.lib.cfqmc_kernel_timing_read_woodbury if woodbury else self.lib.cfqmc_kernel_timing_read
        self._check(fn(self.h, ctypes.byref(a), ctypes.byref(k), ctypes.byref(f)))
        return a.value, k.value, f.value

    def close(self):
        if getattr(self, "h", None) is not None and getattr(self, "_owned", True):
            self.lib.cfqmc_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Heterogeneous batch: one context per group of chains, each on its own stream."""

    def __init__(self, groups):
        """groups: list of dicts of CFQMC keyword arguments (n_phi, l_tau, n_chains, chain_u, ...)."""
        lib = load()
        self.lib = lib
        arr = (Params * len(groups))()
        keep = []
        for k, kw in enumerate(groups):
            p, kp = make_params(**kw)
            arr[k] = p
            keep.extend(kp)
        h = ctypes.c_void_p()
        rc = lib.cfqmc_batch_create(arr, len(groups), ctypes.byref(h))
        if rc != 0:
            raise RuntimeError("cfqmc_batch_create failed: %s" % ERRORS.get(rc, rc))
        self.h = h
        self.groups = []
        for k, kw in enumerate(groups):
            c = ctypes.c_void_p()
            lib.cfqmc_batch_context(h, k, ctypes.byref(c))
            self.groups.append(CFQMC(n_phi=kw.get("n_phi", 6), l_tau=kw.get("l_tau", 40), _handle=c))
        self.n_chains = sum(g.n_chains for g in self.groups)

    def init_fields(self):
        for g in self.groups:
            g.init_fields(None)

    def get(self, chain):
        """(group context view, chain index inside it) of a batch-wide chain index."""
        c, loc = ctypes.c_void_p(), ctypes.c_int32()
        rc = self.lib.cfqmc_batch_get(self.h, chain, ctypes.byref(c), ctypes.byref(loc))
        if rc != 0:
            raise RuntimeError("cfqmc_batch_get failed: %s" % ERRORS.get(rc, rc))
        for g in self.groups:
            if g.h.value == c.value:
                return g, loc.value
        raise RuntimeError("cfqmc_batch_get returned an unknown context")

    def sweep(self, n_sweeps=1, equal_time=False, replay=None):
        """Interleaved sweep of all groups; replay: None or one buffer (or None) per
        group, [n_chains][n_sweeps][l_tau][4 n_q + 1] each (n_sweeps per group)."""
        st = (Stats * self.n_chains)()
        if replay is not None:
            bufs = [None if r is None else np.ascontiguousarray(r, dtype=np.float64) for r in replay]
            ptrs = (ctypes.c_void_p * len(bufs))(*[None if r is None else r.ctypes.data for r in bufs])
            rc = self.lib.cfqmc_batch_sweep_replay(self.h, n_sweeps, ctypes.cast(ptrs, ctypes.c_void_p),
                                                   ctypes.cast(st, ctypes.c_void_p))
        else:
            rc = self.lib.cfqmc_batch_sweep(self.h, n_sweeps, int(bool(equal_time)), ctypes.cast(st, ctypes.c_void_p))
        if rc != 0:
            msgs = []
            for g in self.groups:
                m = self.lib.cfqmc_last_error(g.h)
                if m:
                    msgs.append(m.decode())
            raise RuntimeError("cfqmc_batch_sweep failed: %s (%s)" % (ERRORS.get(rc, rc), "; ".join(msgs)))
        return [s.as_dict() for s in st]

    def close(self):
        if getattr(self, "h", None) is not None:
            for g in self.groups:
                g.h = None
            self.lib.cfqmc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Slmc:
    """Learned global proposal attached to one context (see cfqmc.h)."""

    def __init__(self, ctx, hidden=256, n_qbins=16, n_wbins=16, capacity=10000, max_batch=256, seed=1):
        lib = load()
        self.lib, self.ctx = lib, ctx
        p = SlmcParams()
        lib.cfqmc_slmc_default_params(ctypes.byref(p))
        p.hidden, p.n_qbins, p.n_wbins, p.capacity, p.max_batch, p.seed = (hidden, n_qbins, n_wbins, capacity,
                                                                           max_batch, seed)
        h = ctypes.c_void_p()
        self._check(lib.cfqmc_slmc_create(ctx.h, ctypes.byref(p), ctypes.byref(h)), "create")
        self.h = h
        nf, npar, nd = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        lib.cfqmc_slmc_sizes(h, ctypes.byref(nf), ctypes.byref(npar), ctypes.byref(nd))
        self.n_feat, self.n_params, self.hidden = nf.value, npar.value, hidden
        self.fields_per_chain = ctx.l_tau * 4 * ctx.n_q

    def _check(self, rc, what):
        if rc != 0:
            msg = self.lib.cfqmc_last_error(self.ctx.h)
            raise RuntimeError("cfqmc_slmc_%s failed: %s (%s)" % (what, ERRORS.get(rc, rc),
                                                                 msg.decode() if msg else ""))

    def n_data(self):
        nd = ctypes.c_int32()
        self.lib.cfqmc_slmc_sizes(self.h, None, None, ctypes.byref(nd))
        return nd.value

    def set_params(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        assert w.size == self.n_params
        self._check(self.lib.cfqmc_slmc_set_params(self.h, _ptr(w)), "set_params")

    def get_params(self):
        w = np.empty(self.n_params, dtype=np.float32)
        self._check(self.lib.cfqmc_slmc_get_params(self.h, _ptr(w)), "get_params")
        return w

    def set_norm(self, mu, sigma, y_bar, s_y):
        mu = np.ascontiguousarray(mu, dtype=np.float32)
        sg = np.ascontiguousarray(sigma, dtype=np.float32)
        self._check(self.lib.cfqmc_slmc_set_norm(self.h, _ptr(mu), _ptr(sg), float(y_bar), float(s_y)), "set_norm")

    def get_norm(self):
        mu = np.empty(self.n_feat, dtype=np.float32)
        sg = np.empty(self.n_feat, dtype=np.float32)
        yb, sy = ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.cfqmc_slmc_get_norm(self.h, _ptr(mu), _ptr(sg), ctypes.byref(yb), ctypes.byref(sy)),
                    "get_norm")
        return mu, sg, yb.value, sy.value

    def features(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1, self.fields_per_chain)
        f = np.empty((phi.shape[0], self.n_feat), dtype=np.float32)
        self._check(self.lib.cfqmc_slmc_features(self.h, _ptr(phi), phi.shape[0], _ptr(f)), "features")
        return f

    def action(self, phi, grad=False):
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1, self.fields_per_chain)
        n = phi.shape[0]
        s = np.empty(n)
        g = np.empty_like(phi) if grad else None
        self._check(self.lib.cfqmc_slmc_action(self.h, _ptr(phi), n, _ptr(s), _ptr(g)), "action")
        if grad:
            return s, g.reshape(n, self.ctx.l_tau, 4, self.ctx.n_q)
        return s

    def grad_check(self, phi):
        """(S_NN, dS_NN/dphi) of configurations phi [n][l_tau][4][n_q] from the GPU kernels."""
        phi = np.ascontiguousarray(phi, dtype=np.float64).reshape(-1, self.fields_per_chain)
        n = phi.shape[0]
        f = np.empty(n)
        g = np.empty_like(phi)
        self._check(self.lib.cfqmc_slmc_grad_check(self.h, _ptr(phi), n, _ptr(f), _ptr(g)), "grad_check")
        return f, g.reshape(n, self.ctx.l_tau, 4, self.ctx.n_q)

    def loss_grad(self, x, y):
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float64)
        loss = ctypes.c_double()
        g = np.empty(self.n_params, dtype=np.float32)
        out = np.empty(len(y), dtype=np.float32)
        self._check(self.lib.cfqmc_slmc_loss_grad(self.h, _ptr(x), _ptr(y), len(y), ctypes.byref(loss), _ptr(g),
                                                  _ptr(out)), "loss_grad")
        return loss.value, g, out

    def collect(self):
        self._check(self.lib.cfqmc_slmc_collect(self.h), "collect")

    def clear_data(self):
        self._check(self.lib.cfqmc_slmc_clear_data(self.h), "clear_data")

    def train(self, epochs=10, batch=64, lr=1e-3, refit_norm=False):
        loss = ctypes.c_double()
        self._check(self.lib.cfqmc_slmc_train(self.h, epochs, batch, lr, int(bool(refit_norm)), ctypes.byref(loss)),
                    "train")
        return loss.value

    def train_heldout(self, max_epochs=200, batch=64, lr=1e-3, n_val=256, patience=10, refit_norm=True):
        """Early-stopped training with the last n_val stored configurations held out:
        (last training loss, best validation loss, best epoch)."""
        tl, vl, be = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        self._check(self.lib.cfqmc_slmc_train_heldout(self.h, max_epochs, batch, lr, int(bool(refit_norm)), n_val,
                                                      patience, ctypes.byref(tl), ctypes.byref(vl), ctypes.byref(be)),
                    "train_heldout")
        return tl.value, vl.value, be.value

    SUBSPACES = {"all": 0, "q0": 1, "uniform_q0": 2}

    def set_subspace(self, mode="all"):
        """Global moves on every field ("all"), on component 0 of every channel
        and slice ("q0"), or on the four slice-uniform q = 0 amplitudes
        ("uniform_q0")."""
        self._check(self.lib.cfqmc_slmc_set_subspace(self.h, self.SUBSPACES[mode]), "set_subspace")

    def global_move(self, n_traj=1, n_leap=8, step=0.2, replay=None):
        rp = None if replay is None else np.ascontiguousarray(replay, dtype=np.float64)
        out = (SlmcMove * self.ctx.n_chains)()
        self._check(self.lib.cfqmc_slmc_global_move(self.h, n_traj, n_leap, step, _ptr(rp),
                                                    ctypes.cast(out, ctypes.c_void_p)), "global_move")
        return [m.as_dict() for m in out]

    def last_proposal(self, chain=0):
        out = np.empty((self.ctx.l_tau, 4, self.ctx.n_q))
        self._check(self.lib.cfqmc_slmc_last_proposal(self.h, chain, _ptr(out)), "last_proposal")
        return out

    def close(self):
        if getattr(self, "h", None) is not None:
            self.lib.cfqmc_slmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def green_maxdiff(x, y, stream=None):
    """(return code, [count][2] max|X - Y| and max|X - Y| / max|Y|) of two torch
    complex128 device tensors [count][n][n] by the library's stabilisation check
    (non-finite entries give +inf and CFQMC_ENUMERIC = -4)."""
    lib = load()
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    assert x.shape == y.shape and x.dim() == 3 and x.shape[1] == x.shape[2]
    out = np.empty((x.shape[0], 2))
    rc = lib.cfqmc_green_maxdiff(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), x.shape[1],
                                 x.shape[0], ctypes.c_void_p(stream), _ptr(out))
    return rc, out


def sphere_weights(n_phi):
    """The sphere's density-operator weights n_{l,m}[r, r + m] as a
    [l][m][r] array (N x N x N, zero outside 0 <= m <= l, r + m < N)."""
    lib = load()
    out = np.zeros((n_phi, n_phi, n_phi))
    rc = lib.cfqmc_sphere_weights(int(n_phi), _ptr(out))
    if rc != 0:
        raise RuntimeError("cfqmc_sphere_weights failed: %s" % ERRORS.get(rc, rc))
    return out

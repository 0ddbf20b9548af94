"""Recorded Markov-chain histories of the FP64 oracle at the workload shapes.

Writes tests/golden/hist_<name>.npz for the GPU replay tests. Only the oracle
(oracle/) and the seeded input generators (synth/) are used: the initial
fields and the replayed proposal noise are regenerated from the seeds stored
in each file, and every stored value is an oracle output.

Shapes (torus unless noted; fields N(0, 1); one Langevin proposal per slice, Methods,
Langevin-based global update scheme, adaptive step on):
  c2_n36   N_phi = 36, |q| l_B <= 3 (161 components), L = 200, dtau = 0.1,
           five chains at u = 0.5, 1.0, 1.5, 2.0, 2.5, one sweep each
  c3_n100  N_phi = 100, paper cutoff (933), u = 1.5, on a 16-slice axis,
           two sweeps
  c4_n24, c4_n48, c4_n72
           N_phi = 24 / 48 / 72, paper cutoff (221 / 437 / 665) on 12-slice
           axes, u = 0.5, 1.667, 3.0 (ends and middle of the 16-point grid
           0.5 + j / 6), one sweep each
  c5_n140  N_phi = 140, paper cutoff (1305), u = 1.5, 8-slice axis, one sweep
  sphere_n59
           the paper's largest sphere, N_phi = 59 (3481 components per channel),
           dtau = 0.01, u = 0.2, 8-slice axis, n_stab = 4, one sweep at eps = 0.05
           (the sphere's larger exponents need a smaller Langevin step)

Usage: python tests/golden/make_histories.py [name ...]   (default: all)
Per chain the file holds: acc<k> [sweeps][L] accept flags, lna<k> ln A,
eps<k> the step after each sweep, phi<k> the final fields [L][4][n_q],
G<k> and Gm<k> the spin-block G(0) and G(L/2) of the final fields, ld<k> ln w_F.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import dqmc  # noqa: E402
from oracle.model import Model, Q_PAPER, Q_RADIUS, Q_SPHERE  # noqa: E402

CONFIGS = {
    "c2_n36": dict(n_phi=36, l_tau=200, dtau=0.1, q_mode=Q_RADIUS, q_max=3.0, u=[0.5, 1.0, 1.5, 2.0, 2.5],
                   n_stab=10, n_sweeps=1, eps0=0.4, seed_f=21, seed_r=121),
    "c3_n100": dict(n_phi=100, l_tau=16, dtau=0.1, q_mode=Q_PAPER, q_max=None, u=[1.5], n_stab=8, n_sweeps=2,
                    eps0=0.4, seed_f=3, seed_r=103),
    "c4_n24": dict(n_phi=24, l_tau=12, dtau=0.1, q_mode=Q_PAPER, q_max=None, u=[0.5], n_stab=10, n_sweeps=1,
                   eps0=0.4, seed_f=400, seed_r=500),
    "c4_n48": dict(n_phi=48, l_tau=12, dtau=0.1, q_mode=Q_PAPER, q_max=None, u=[0.5 + 7 / 6], n_stab=10,
                   n_sweeps=1, eps0=0.4, seed_f=416, seed_r=516),
    "c4_n72": dict(n_phi=72, l_tau=12, dtau=0.1, q_mode=Q_PAPER, q_max=None, u=[3.0], n_stab=10, n_sweeps=1,
                   eps0=0.4, seed_f=432, seed_r=532),
    "c5_n140": dict(n_phi=140, l_tau=8, dtau=0.1, q_mode=Q_PAPER, q_max=None, u=[1.5], n_stab=4, n_sweeps=1,
                    eps0=0.4, seed_f=5, seed_r=105),
    "sphere_n59": dict(n_phi=59, l_tau=8, dtau=0.01, q_mode=Q_SPHERE, q_max=None, u=[0.2], n_stab=4, n_sweeps=1,
                       eps0=0.05, seed_f=59, seed_r=159, exp_squarings=10),
}


def inputs(cfg, k, n_q):
    """Initial fields and replay buffer of chain k (seeded, shared with the GPU tests)."""
    phi = synth.fields(cfg["seed_f"] + k, cfg["l_tau"], n_q)
    rp = synth.replay(cfg["seed_r"] + k, cfg["n_sweeps"], cfg["l_tau"], n_q)
    return phi, rp


def model(cfg, u):
    return Model(cfg["n_phi"], cfg["l_tau"], cfg["dtau"], u0=1.0, uk=u, un=u, q_mode=cfg["q_mode"],
                 q_max=cfg["q_max"])


def make(name):
    cfg = CONFIGS[name]
    L = cfg["l_tau"]
    out = {"meta_json": np.array(json.dumps(cfg))}
    for k, u in enumerate(cfg["u"]):
        m = model(cfg, u)
        phi, rp = inputs(cfg, k, m.n_q)
        ch = dqmc.Chain(m, phi, eps0=cfg["eps0"], adapt=True)
        acc, lna, eps = [], [], []
        t0 = time.time()
        for s in range(cfg["n_sweeps"]):
            ch.sweep(rp[s])
            hist = ch.history[-L:]
            acc.append([int(h[2]) for h in hist])
            lna.append([h[1] for h in hist])
            eps.append(ch.eps)
        Bs = dqmc.propagators(m, ch.phi)
        out["acc%d" % k] = np.array(acc, dtype=np.int8)
        out["lna%d" % k] = np.array(lna)
        out["eps%d" % k] = np.array(eps)
        out["phi%d" % k] = ch.phi
        out["G%d" % k] = dqmc.green(m, ch.phi, 0, Bs)
        out["Gm%d" % k] = dqmc.green(m, ch.phi, L // 2, Bs)
        out["ld%d" % k] = np.array(dqmc.logdet(m, ch.phi, Bs))
        print("%s chain %d: n_q %d, accepted %d of %d, %.1f s" % (name, k, m.n_q, int(np.sum(acc)),
                                                                 L * cfg["n_sweeps"], time.time() - t0),
              flush=True)
    np.savez_compressed(os.path.join(HERE, "hist_%s.npz" % name), **out)


if __name__ == "__main__":
    names = sys.argv[1:] or list(CONFIGS)
    for nm in names:
        make(nm)

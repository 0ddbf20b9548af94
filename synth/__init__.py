"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the method: it only draws random numbers.
Everything the Monte Carlo method consumes as randomness (initial fields,
Gaussian proposal noise, uniform acceptance draws) is produced here and
handed to both sides as plain arrays.

Layouts (all float64, C order):
  fields         [l_tau][4][n_q]          auxiliary fields, one set per channel
  replay buffer  [n_sweeps][l_tau][4*n_q+1]  per slice: 4*n_q normals, then u
"""
import numpy as np


def fields(seed, l_tau, n_q, scale=1.0):
    """Initial auxiliary fields drawn i.i.d. N(0, scale^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return scale * rng.standard_normal((l_tau, 4, n_q))


def replay(seed, n_sweeps, l_tau, n_q):
    """Proposal noise and acceptance uniforms for n_sweeps sweeps.

    Returns an array [n_sweeps][l_tau][4*n_q+1]: entries 0..4*n_q-1 of a slice
    are the standard normals eta (channel-major: channel*n_q + component), the
    last entry is the uniform u in [0, 1).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((n_sweeps, l_tau, 4 * n_q + 1))
    out[..., :4 * n_q] = rng.standard_normal((n_sweeps, l_tau, 4 * n_q))
    out[..., 4 * n_q] = rng.random((n_sweeps, l_tau))
    return out


def mlp_batch(seed, n, dim, scale=1.0):
    """Random feature batch for network gradient checks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return scale * rng.standard_normal((n, dim))

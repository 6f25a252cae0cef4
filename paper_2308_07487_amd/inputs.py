"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method: it only draws positions and
spin frames (numpy, seeded) with the shapes and distributions of the
workloads.  Both the GPU path and the CPU oracle consume what it returns.

Workload recipes (lattice constant 1, unit spins, fp32 xyz):

- ``sc_positions(L)``: simple-cubic periodic lattice, sites at integer points.
- ``bcc_positions(L)``: body-centred cubic, corners n and centres n + 1/2.
- ``ball_positions(n, R, seed)``: n points uniform in a ball of radius R.
- ``random_unit_frames``: independent uniform unit vectors per site and frame.
- ``axis_frames``: random signed axis vectors (|S|^2 = 1 exactly in fp32).
- ``dyadic_frames``: components on the grid (1/16) Z, not normalised, so
  that every product and every partial sum up to 2^24 units is exact in FP32.
- ``static_frames``: every spin along one fixed axis in every frame.
- ``spiral_frames``: a planted spin wave with a commensurate wave vector.
- ``powder_wave_vectors``: wave vectors with random directions and a range
  of magnitudes, for q-resolved spectra of samples without a lattice.
- ``batch_samples``: the recipe of a batch of independent samples (lattice,
  box edge, origin and lag counts, seeds), as the paper's averages over many
  realizations of different lattices need.
"""
from __future__ import annotations

import numpy as np


def sc_positions(L):
    L = _dims(L)
    g = np.stack(np.meshgrid(np.arange(L[0]), np.arange(L[1]), np.arange(L[2]), indexing="ij"),
                 axis=-1)
    return g.reshape(-1, 3).astype(np.float32)


def bcc_positions(L):
    c = sc_positions(L)
    b = c + np.float32(0.5)
    out = np.empty((2 * c.shape[0], 3), dtype=np.float32)
    out[0::2] = c
    out[1::2] = b
    return out


def ball_positions(n, R, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = R * rng.random(n) ** (1.0 / 3.0)
    return (v * r[:, None]).astype(np.float32)


def random_unit_frames(n_frames, n, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n_frames, n, 3))
    v /= np.linalg.norm(v, axis=2, keepdims=True)
    return v.astype(np.float32)


def axis_frames(n_frames, n, seed):
    """Random signed unit axis vectors: the only fp32 unit vectors whose
    squared length is exactly 1."""
    rng = np.random.default_rng(seed)
    out = np.zeros((n_frames, n, 3), dtype=np.float32)
    a = rng.integers(0, 3, size=(n_frames, n))
    sgn = rng.choice(np.array([-1.0, 1.0], dtype=np.float32), size=(n_frames, n))
    np.put_along_axis(out, a[..., None], sgn[..., None], axis=2)
    return out


def dyadic_frames(n_frames, n, seed):
    rng = np.random.default_rng(seed)
    return (rng.integers(-16, 17, size=(n_frames, n, 3)) / 16.0).astype(np.float32)


def static_frames(n_frames, n, axis):
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    return np.broadcast_to(a.astype(np.float32), (n_frames, n, 3)).copy()


def spiral_frames(pos, q, theta, omega, n_frames, dt):
    """S_i(f) = (sin th cos phi, sin th sin phi, cos th), phi = q.r_i - omega f dt."""
    pos = np.asarray(pos, dtype=np.float64)
    t = np.arange(n_frames, dtype=np.float64)[:, None] * dt
    phi = pos @ np.asarray(q, dtype=np.float64) - omega * t
    s, c = np.sin(theta), np.cos(theta)
    out = np.stack([s * np.cos(phi), s * np.sin(phi), np.full_like(phi, c)], axis=-1)
    return out.astype(np.float32)


def batch_samples(n_samples=48, seed=0x5DC00500, edge=(10, 40), origins=(32, 128), lags=(64, 256)):
    """Sample m: sc for even m, bcc for odd m; cubic box edge uniform in
    `edge` (the first sample takes the smallest edge, the last the largest),
    origin and lag counts uniform in `origins` and `lags`, trajectory seed
    seed + m.  Returns a list of dicts (lattice, cells, n_origins, n_lags, seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for m in range(n_samples):
        L = int(rng.integers(edge[0], edge[1] + 1))
        if m == 0:
            L = edge[0]
        elif m == n_samples - 1:
            L = edge[1]
        out.append(dict(lattice="sc" if m % 2 == 0 else "bcc", cells=(L, L, L),
                        n_origins=int(rng.integers(origins[0], origins[1] + 1)),
                        n_lags=int(rng.integers(lags[0], lags[1] + 1)), seed=seed + m))
    return out


def permute_sites(pos, frames, seed):
    """Same sample with the site order shuffled (positions and frames together)."""
    p = np.random.default_rng(seed).permutation(pos.shape[0])
    return pos[p].copy(), frames[:, p].copy(), p


def _dims(L):
    if np.isscalar(L):
        return (int(L),) * 3
    return tuple(int(x) for x in L)


def powder_wave_vectors(n_q, q_min, q_max, seed):
    """n_q wave vectors with directions uniform on the sphere and magnitudes
    uniform in [q_min, q_max] (radians per unit length), for samples without
    a reciprocal lattice."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n_q, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v * rng.uniform(q_min, q_max, size=(n_q, 1))

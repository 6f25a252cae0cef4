"""FP64 CPU oracle for the binned spin pair correlation (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
nothing here imports the product package.

The arithmetic lives in ``sdc_oracle.c`` (plain C, FP64, OpenMP over the
origin site i); this module loads it with ctypes and converts numpy arrays.
Each function states the paper passage it follows (arXiv 2308.07487):

- ``binned_corr``      Eq. (4) unsubtracted, summed over alpha as in Eq. (3),
                       cast per lag as the GEMM of Sec. 3.2 and binned by a
                       key computed from positions (the role of Q in Eq. (6));
                       with ``connected=True`` the second term of Eq. (4), the
                       product of the per-site averages over the origins
                       (``mean_product``), is subtracted.
- ``structure_factor_q`` Eq. (3), the double sum over site pairs written out,
                       at any wave vector (``structure_factor``: the ones
                       commensurate with a periodic box); ``connected`` takes
                       Eq. (4) with its second term.
- ``binned_corr_fft``  the same H on periodic lattices through the
                       correlation theorem (numpy FFT): a special case that
                       reduces to a library routine, pinned against
                       ``binned_corr``, for checks of every bin and lag at the
                       workloads' full sizes.
- ``finalize``         per-bin normalisation, site sum (Sec. 1: summing the
                       correlation over all sites) and the windowed time
                       transform of Sec. 2.2.
- ``ll_rk4``           Eq. (2) with the Hamiltonian of Eq. (1) (exchange, DMI,
                       single-ion anisotropy, field), RK4 without
                       renormalisation (Sec. 3.1).
- ``mc_anneal``        Metropolis Monte Carlo with a cone of trial moves
                       adapted to the acceptance rate (Sec. 2.1) and
                       simulated annealing (Sec. 4.3) on the Hamiltonian of
                       Eq. (1); greedy colour classes updated in turn.
- ``philox`` / ``init_state``  Philox4x32-10 (Salmon et al., SC'11) seeded
                       initial states.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sdc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libsdc_oracle.so")

SC, BCC, RADIAL = 0, 1, 2
_ERR = {1: "invalid argument", 3: "out of memory"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
            "-std=c11", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm",
        ])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, f32, f64, u64, u32 = (ctypes.c_int64, ctypes.c_int32, ctypes.c_float,
                                         ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32)
        L.oracle_n_bins.argtypes = [P, i64, ctypes.c_int, P, i32, f32, P]
        L.oracle_pair_keys.argtypes = [P, i64, ctypes.c_int, P, i32, f32, P, P, i64, P]
        L.oracle_binned_corr.argtypes = [P, i64, ctypes.c_int, P, i32, f32, P, i64, i32, i32,
                                         P, i32, i64, i64, P, P, ctypes.c_int]
        L.oracle_binned_corr_select.argtypes = [P, i64, ctypes.c_int, P, i32, f32, P, i64, i32,
                                                i32, P, i32, P, i32, P, P, ctypes.c_int]
        L.oracle_self_corr.argtypes = [P, i64, i64, i32, i32, P, i32, P]
        L.oracle_mean_product.argtypes = [P, i64, ctypes.c_int, P, i32, f32, P, i64, i32, i32,
                                          P, i32, i64, i64, P, i32, P, ctypes.c_int]
        L.oracle_self_mean_product.argtypes = [P, i64, i64, i32, i32, P, i32, P]
        L.oracle_dft.argtypes = [P, i32, P]
        L.oracle_finalize.argtypes = [P, P, i64, i32, i64, P, P, P, P, P, P, P]
        L.oracle_ll_rk4.argtypes = [i64, P, P, P, P, f64, i64, P]
        L.oracle_ll_rk4_full.argtypes = [i64, P, P, P, P, f64, f64, P, f64, i64, P]
        L.oracle_mc_n_sweeps.argtypes = [f64, f64, f64, i64, i64, P]
        L.oracle_mc_anneal.argtypes = [i64, P, P, P, P, f64, f64, u64, f64, f64, f64, i64, i64, f64, f64,
                                       P, P, P, P, ctypes.c_int]
        L.oracle_philox.argtypes = [u64, u32, i64, i64, P]
        L.oracle_init_state.argtypes = [u64, i64, ctypes.c_int, f64, P]
        L.oracle_philox_block.argtypes = [P, P, P]
        for name in ("oracle_n_bins", "oracle_pair_keys", "oracle_binned_corr",
                     "oracle_binned_corr_select", "oracle_self_corr", "oracle_dft",
                     "oracle_finalize", "oracle_ll_rk4", "oracle_ll_rk4_full", "oracle_philox",
                     "oracle_init_state", "oracle_mc_n_sweeps", "oracle_mc_anneal",
                     "oracle_philox_block", "oracle_mean_product", "oracle_self_mean_product"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what}: {_ERR.get(rc, rc)}")


def _spec(kind, cells, n_shells, r_max):
    cells = np.ascontiguousarray(cells if cells is not None else (0, 0, 0), dtype=np.int32)
    return int(kind), cells, int(n_shells), float(r_max)


def n_bins(pos, kind, cells=None, n_shells=0, r_max=0.0):
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    kind, cells, n_shells, r_max = _spec(kind, cells, n_shells, r_max)
    out = ctypes.c_int64(0)
    _check(lib().oracle_n_bins(_ptr(pos), pos.shape[0], kind, _ptr(cells), n_shells, r_max,
                               ctypes.byref(out)), "n_bins")
    return int(out.value)


def pair_keys(pos, kind, pi, pj, cells=None, n_shells=0, r_max=0.0):
    """Bin of each ordered pair (pi[p] = origin site, pj[p] = later site)."""
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    kind, cells, n_shells, r_max = _spec(kind, cells, n_shells, r_max)
    pi = np.ascontiguousarray(pi, dtype=np.int64)
    pj = np.ascontiguousarray(pj, dtype=np.int64)
    out = np.zeros(pi.shape[0], dtype=np.int64)
    _check(lib().oracle_pair_keys(_ptr(pos), pos.shape[0], kind, _ptr(cells), n_shells, r_max,
                                  _ptr(pi), _ptr(pj), pi.shape[0], _ptr(out)), "pair_keys")
    return out


def binned_corr(pos, frames, kind, n_origins, lags, stride=1, cells=None, n_shells=0,
                r_max=0.0, rows=None, counts=True, n_threads=0, connected=False):
    """Raw binned sums H[l][b] (FP64) and pair counts (uint64).

    H[l][b] = sum over ordered pairs (i, j) with key(i, j) = b of
              sum_{o < n_origins} S_i(o*stride) . S_j(o*stride + lags[l]).
    ``rows`` = (i_begin, i_end) restricts the origin sites (partial sums).
    ``connected``: subtract ``mean_product`` (Eq. (4), second term).
    """
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    frames = np.ascontiguousarray(frames, dtype=np.float32)
    n = pos.shape[0]
    assert frames.ndim == 3 and frames.shape[1] == n and frames.shape[2] == 3
    kind_, cells_, ns, rm = _spec(kind, cells, n_shells, r_max)
    nb = n_bins(pos, kind, cells, n_shells, r_max)
    lags = np.ascontiguousarray(lags, dtype=np.int32)
    i0, i1 = (0, n) if rows is None else rows
    H = np.zeros((lags.shape[0], nb), dtype=np.float64)
    C = np.zeros(nb, dtype=np.uint64) if counts else None
    _check(lib().oracle_binned_corr(_ptr(pos), n, kind_, _ptr(cells_), ns, rm, _ptr(frames),
                                    frames.shape[0], int(n_origins), int(stride), _ptr(lags),
                                    lags.shape[0], int(i0), int(i1), _ptr(H), _ptr(C),
                                    int(n_threads)), "binned_corr")
    if connected:
        H -= mean_product(pos, frames, kind, n_origins, lags, stride=stride, cells=cells,
                          n_shells=n_shells, r_max=r_max, rows=rows, n_threads=n_threads)
    return H, C


def _fast_len(n):
    """Smallest 2^a 3^b 5^c >= n (an FFT length numpy handles quickly)."""
    m = n
    while True:
        r = m
        for f in (2, 3, 5):
            while r % f == 0:
                r //= f
        if r == 1:
            return m
        m += 1


def binned_corr_fft(pos, frames, kind, n_origins, lags, cells, stride=1):
    """H[l][b] of ``binned_corr`` for the periodic kinds through the
    correlation theorem (numpy FFT, FP64), for checks of every bin and lag at
    sizes the double loop cannot reach.

    On a periodic lattice the bin of a pair is the displacement class, so
    H(d, t) = sum_o sum_x sum_alpha S_alpha(o s, x) S_alpha(o s + t, x + d),
    a cross-correlation over the periodic site grid and, with the origin
    frames o s kept and every other frame zeroed on the origin side, over
    time as well: one 4D correlation per component, conj(F[A]) F[B] in
    Fourier space (A real).  The time axis is zero-padded past
    (n_origins - 1) s + max lag, so no lag wraps around.  bcc is two
    interleaved sc grids: parity-0 bins take the same-sublattice
    correlations, parity-1 bins the corner-to-centre one plus the
    centre-to-corner one shifted by a cell (its key subtracts (1,1,1)).
    Pinned against ``binned_corr`` (tests/test_oracle.py)."""
    if kind not in (SC, BCC):
        raise ValueError("binned_corr_fft needs a periodic kind")
    L = tuple(int(c) for c in cells)
    p = np.asarray(pos, dtype=np.float64)
    f = np.asarray(frames)
    n = p.shape[0]
    if kind == SC:
        cell = np.rint(p).astype(np.int64) % np.array(L)
        beta = np.zeros(n, dtype=np.int64)
    else:
        d = np.rint(2.0 * p).astype(np.int64)
        beta = d[:, 0] % 2
        cell = ((d - beta[:, None]) // 2) % np.array(L)
    flat = (cell[:, 0] * L[1] + cell[:, 1]) * L[2] + cell[:, 2]
    lags = np.asarray(lags, dtype=np.int64)
    need = (n_origins - 1) * stride + int(lags.max()) + 1
    if need > f.shape[0]:
        raise ValueError("not enough frames for the origins and lags")
    P = _fast_len(need)
    ncell = L[0] * L[1] * L[2]
    orig = np.arange(n_origins) * stride
    nsub = 1 if kind == SC else 2
    shape = (P,) + L
    X = {}
    for a in range(3):
        FA, FB = [], []
        for b in range(nsub):
            sites = np.nonzero(beta == b)[0]
            G = np.zeros((P, ncell))
            G[orig[:, None], flat[sites][None, :]] = f[orig][:, sites, a]
            FA.append(np.fft.rfftn(G.reshape(shape), axes=(0, 1, 2, 3)))
            G = np.zeros((P, ncell))
            G[:need, flat[sites]] = f[:need][:, sites, a]
            FB.append(np.fft.rfftn(G.reshape(shape), axes=(0, 1, 2, 3)))
            del G
        for (u, v) in ([(0, 0)] if nsub == 1 else [(0, 0), (1, 1), (0, 1), (1, 0)]):
            key = (0, 0) if u == v else (u, v)
            term = np.conj(FA[u]) * FB[v]
            X[key] = X[key] + term if key in X else term
    axes = (0, 1, 2, 3)
    h0 = np.fft.irfftn(X[(0, 0)], s=shape, axes=axes)[lags].reshape(len(lags), ncell)
    if nsub == 1:
        return h0
    h1 = np.fft.irfftn(X[(0, 1)], s=shape, axes=axes)[lags]
    h1 += np.roll(np.fft.irfftn(X[(1, 0)], s=shape, axes=axes)[lags], shift=(-1, -1, -1), axis=(1, 2, 3))
    H = np.empty((len(lags), 2 * ncell))
    H[:, 0::2] = h0
    H[:, 1::2] = h1.reshape(len(lags), ncell)
    return H


def mean_product(pos, frames, kind, n_origins, lags, stride=1, cells=None, n_shells=0,
                 r_max=0.0, rows=None, bins=None, n_threads=0):
    """Second term of Eq. (4), binned like ``binned_corr``:
    P[l][b] = n_origins * sum over ordered pairs (i, j) with key(i, j) = b of
              <S_i(t0)> . <S_j(t0 + lags[l])>, <.> = average over t0 = o*stride.
    ``bins``: only these bins (P is then [n_lags][len(bins)])."""
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    frames = np.ascontiguousarray(frames, dtype=np.float32)
    n = pos.shape[0]
    kind_, cells_, ns, rm = _spec(kind, cells, n_shells, r_max)
    lags = np.ascontiguousarray(lags, dtype=np.int32)
    i0, i1 = (0, n) if rows is None else rows
    if bins is None:
        width, bp, nsel = n_bins(pos, kind, cells, n_shells, r_max), None, 0
    else:
        bins = np.ascontiguousarray(bins, dtype=np.int64)
        width, bp, nsel = bins.shape[0], _ptr(bins), bins.shape[0]
    P = np.zeros((lags.shape[0], width), dtype=np.float64)
    _check(lib().oracle_mean_product(_ptr(pos), n, kind_, _ptr(cells_), ns, rm, _ptr(frames),
                                     frames.shape[0], int(n_origins), int(stride), _ptr(lags),
                                     lags.shape[0], int(i0), int(i1), bp, int(nsel), _ptr(P),
                                     int(n_threads)), "mean_product")
    return P


def binned_corr_select(pos, frames, kind, n_origins, lags, bins, stride=1, cells=None,
                       n_shells=0, r_max=0.0, n_threads=0, connected=False):
    """H restricted to selected bins: returns (H_sel[n_lags][n_sel], counts_sel)."""
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    frames = np.ascontiguousarray(frames, dtype=np.float32)
    kind_, cells_, ns, rm = _spec(kind, cells, n_shells, r_max)
    lags = np.ascontiguousarray(lags, dtype=np.int32)
    bins = np.ascontiguousarray(bins, dtype=np.int64)
    H = np.zeros((lags.shape[0], bins.shape[0]), dtype=np.float64)
    C = np.zeros(bins.shape[0], dtype=np.uint64)
    _check(lib().oracle_binned_corr_select(_ptr(pos), pos.shape[0], kind_, _ptr(cells_), ns, rm,
                                           _ptr(frames), frames.shape[0], int(n_origins),
                                           int(stride), _ptr(lags), lags.shape[0], _ptr(bins),
                                           bins.shape[0], _ptr(H), _ptr(C), int(n_threads)),
           "binned_corr_select")
    if connected:
        H -= mean_product(pos, frames, kind, n_origins, lags, stride=stride, cells=cells,
                          n_shells=n_shells, r_max=r_max, bins=bins, n_threads=n_threads)
    return H, C


def self_corr(frames, n_origins, lags, stride=1, connected=False):
    """sum_o sum_i S_i(o*stride) . S_i(o*stride + lag), per lag (FP64); with
    ``connected`` minus n_origins * sum_i <S_i(t0)> . <S_i(t0 + lag)>."""
    frames = np.ascontiguousarray(frames, dtype=np.float32)
    lags = np.ascontiguousarray(lags, dtype=np.int32)
    out = np.zeros(lags.shape[0], dtype=np.float64)
    _check(lib().oracle_self_corr(_ptr(frames), frames.shape[1], frames.shape[0], int(n_origins),
                                  int(stride), _ptr(lags), lags.shape[0], _ptr(out)), "self_corr")
    if connected:
        mp = np.zeros(lags.shape[0], dtype=np.float64)
        _check(lib().oracle_self_mean_product(_ptr(frames), frames.shape[1], frames.shape[0],
                                              int(n_origins), int(stride), _ptr(lags), lags.shape[0],
                                              _ptr(mp)), "self_mean_product")
        out -= mp
    return out


def structure_factor(pos, frames, n_origins, lags, m, cells, stride=1):
    """Eq. (3) at the wave vectors commensurate with a periodic box,
    q_a = 2 pi m_a / L_a (``structure_factor_q`` with those q).
    Returns complex128 [n_q][n_lags]."""
    m = np.atleast_2d(np.asarray(m, dtype=np.float64))
    L = np.asarray(cells, dtype=np.float64)
    return structure_factor_q(pos, frames, n_origins, lags, 2.0 * np.pi * m / L, stride=stride)


def structure_factor_q(pos, frames, n_origins, lags, q, stride=1, connected=False):
    """Eq. (3) written out at arbitrary wave vectors q (rows of [n_q][3]):
    S(q, t) = (1 / (N n_o)) sum_o sum_i sum_j exp(-i q.(r_j - r_i)) S_i(o s) . S_j(o s + t),
    the double sum over all ordered site pairs with the actual positions r
    (no periodic image), site j at the later time.  ``connected`` subtracts
    the second term of Eq. (4): n_o <S_i(t0)> . <S_j(t0 + t)> per pair, <.>
    the average over the origins t0 = o s.  numpy, FP64; the per-origin pair
    matrix is a matrix product.  Returns complex128 [n_q][n_lags]."""
    pos = np.asarray(pos, dtype=np.float64)
    f = np.asarray(frames, dtype=np.float64)
    n = pos.shape[0]
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    out = np.zeros((q.shape[0], len(lags)), dtype=np.complex128)
    org = np.arange(n_origins) * stride
    for li, t in enumerate(lags):
        G = np.zeros((n, n))
        for o in org:
            G += f[o] @ f[o + t].T  # G[i, j] = S_i(o s) . S_j(o s + t)
        if connected:
            G -= n_origins * (f[org].mean(axis=0) @ f[org + t].mean(axis=0).T)
        for qi in range(q.shape[0]):
            phase = np.exp(-1j * (pos @ q[qi]))          # exp(-i q.r)
            P = np.conj(phase)[:, None] * phase[None, :]  # exp(-i q.(r_j - r_i))
            out[qi, li] = np.sum(P * G) / (n * n_origins)
    return out


def dft(x):
    """Half-Hann windowed DFT, complex128."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros((x.shape[0], 2), dtype=np.float64)
    _check(lib().oracle_dft(_ptr(x), x.shape[0], _ptr(out)), "dft")
    return out[:, 0] + 1j * out[:, 1]


def finalize(H, counts, n_sites, n_org, self_raw):
    """C[l][b], Csum[l], Cself[l], Ssum[k] (complex), Sself[k] (complex)."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    nl, nb = H.shape
    n_org = np.ascontiguousarray(np.broadcast_to(np.asarray(n_org, dtype=np.float64), (nl,)))
    self_raw = np.ascontiguousarray(self_raw, dtype=np.float64)
    C = np.zeros_like(H)
    Cs = np.zeros(nl)
    Cf = np.zeros(nl)
    Ss = np.zeros((nl, 2))
    Sf = np.zeros((nl, 2))
    _check(lib().oracle_finalize(_ptr(H), _ptr(counts), nb, nl, int(n_sites), _ptr(n_org),
                                 _ptr(self_raw), _ptr(C), _ptr(Cs), _ptr(Cf), _ptr(Ss), _ptr(Sf)),
           "finalize")
    return C, Cs, Cf, Ss[:, 0] + 1j * Ss[:, 1], Sf[:, 0] + 1j * Sf[:, 1]


def ll_rk4(row, col, J, init, dt, n_frames, D=None, A=0.0, Hz=0.0):
    """RK4 frames [n_frames][n][3] (FP64) for Eq. (2) with the Hamiltonian of
    Eq. (1): dS_i/dt = h_i x S_i, h_i = sum_j (J_ij S_j + D_ij x S_j)
    - 2 A S_i^z z - H_z z.  CSR bonds (row, col, J); D: [nnz][3] DMI vectors of
    the ordered pairs (D_ji = -D_ij) or None."""
    row = np.ascontiguousarray(row, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    J = np.ascontiguousarray(J, dtype=np.float64)
    init = np.ascontiguousarray(init, dtype=np.float32)
    n = init.shape[0]
    out = np.zeros((int(n_frames), n, 3), dtype=np.float64)
    Dp = None
    if D is not None:
        D = np.ascontiguousarray(D, dtype=np.float64).reshape(-1, 3)
        assert D.shape[0] == col.shape[0]
        Dp = _ptr(D)
    _check(lib().oracle_ll_rk4_full(n, _ptr(row), _ptr(col), _ptr(J), Dp, float(A), float(Hz), _ptr(init),
                                    float(dt), int(n_frames), _ptr(out)), "ll_rk4")
    return out


def mc_n_sweeps(T_start, T_end, cool, sweeps_per_T, sweeps_final):
    """Sweeps of the annealing schedule (T_k = T_start cool^k while T_k > T_end,
    sweeps_per_T each, then sweeps_final at T_end)."""
    n = ctypes.c_int64()
    _check(lib().oracle_mc_n_sweeps(float(T_start), float(T_end), float(cool), int(sweeps_per_T),
                                    int(sweeps_final), ctypes.byref(n)), "mc_n_sweeps")
    return int(n.value)


def mc_anneal(row, col, J, init, seed, T_start, T_end, cool, sweeps_per_T, sweeps_final,
              cone0=np.pi, acc_target=0.2, D=None, A=0.0, Hz=0.0, site_order=False):
    """Annealed Metropolis sweeps with an adaptive cone (Sec. 2.1, Sec. 4.3) on
    CSR bonds with the Hamiltonian of Eq. (1).  Sweeps visit the greedy colour
    classes in turn (the order a parallel sweep reproduces move for move), or
    with ``site_order`` the sites in plain index order (the sequential sweep).
    Returns (state [n][3] FP64, accepted moves per sweep, energy per site,
    final cone, last T, colour classes visited)."""
    row = np.ascontiguousarray(row, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    J = np.ascontiguousarray(J, dtype=np.float64)
    init = np.ascontiguousarray(init, dtype=np.float32)
    n = init.shape[0]
    ns = mc_n_sweeps(T_start, T_end, cool, sweeps_per_T, sweeps_final)
    state = np.zeros((n, 3))
    acc = np.zeros(max(ns, 1), dtype=np.int64)
    info = np.zeros(4)
    Dp = None
    if D is not None:
        D = np.ascontiguousarray(D, dtype=np.float64).reshape(-1, 3)
        assert D.shape[0] == col.shape[0]
        Dp = _ptr(D)
    _check(lib().oracle_mc_anneal(n, _ptr(row), _ptr(col), _ptr(J), Dp, float(A), float(Hz), int(seed),
                                  float(T_start), float(T_end), float(cool), int(sweeps_per_T),
                                  int(sweeps_final), float(cone0), float(acc_target), _ptr(init),
                                  _ptr(state), _ptr(acc), _ptr(info), int(bool(site_order))), "mc_anneal")
    return state, acc[:ns], float(info[0]), float(info[1]), float(info[2]), int(info[3])


def philox(seed, draw, idx0, n_blocks):
    out = np.zeros((int(n_blocks), 4), dtype=np.uint32)
    _check(lib().oracle_philox(int(seed), int(draw), int(idx0), int(n_blocks), _ptr(out)), "philox")
    return out


def philox_block(ctr, key):
    """One raw Philox4x32-10 block for a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _check(lib().oracle_philox_block(_ptr(c), _ptr(k), _ptr(out)), "philox_block")
    return out


def init_state(seed, n, mode=0, sigma=0.0):
    out = np.zeros((int(n), 3), dtype=np.float64)
    _check(lib().oracle_init_state(int(seed), int(n), int(mode), float(sigma), _ptr(out)),
           "init_state")
    return out

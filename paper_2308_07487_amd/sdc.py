"""Python binding of the sdc C ABI (include/sdc.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels; this module
converts numpy arrays and torch device tensors to pointers, calls the entry
points with the same names, and turns status codes into exceptions.  torch is
used only for device memory and streams.  If the compiled library is missing
the import fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdc.so")

OK, ERR_INVALID_ARG, ERR_STATE, ERR_OOM, ERR_HIP, ERR_UNSUPPORTED, ERR_NO_DEVICE = range(7)
PREC_FP32, PREC_SPLIT_BF16, PREC_SPLIT_FP16, PREC_BF16X3 = 0, 1, 2, 3
BINS_SC, BINS_BCC, BINS_RADIAL = 0, 1, 2
COUPLING_NN_UNIFORM, COUPLING_NN_RANDOM_SIGN, COUPLING_EXP_CUTOFF = 0, 1, 2
INIT_UNIFORM, INIT_PERTURBED_Z, INIT_GIVEN = 0, 1, 2

PRECISIONS = {"fp32": PREC_FP32, "split_bf16": PREC_SPLIT_BF16, "split_fp16": PREC_SPLIT_FP16,
              "bf16x3": PREC_BF16X3}


class SdcError(RuntimeError):
    def __init__(self, status, what, detail):
        super().__init__(f"{what}: {status_string(status)} ({detail})")
        self.status = status


class BinSpec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("cells", ctypes.c_int32 * 3),
                ("n_shells", ctypes.c_int32), ("r_max", ctypes.c_float)]


class CorrSpec(ctypes.Structure):
    _fields_ = [("n_origins", ctypes.c_int32), ("n_lags", ctypes.c_int32),
                ("origin_stride", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class McSpec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("cells", ctypes.c_int32 * 3), ("coupling", ctypes.c_int32),
                ("r_cut", ctypes.c_float), ("J", ctypes.c_double), ("D", ctypes.c_double),
                ("A", ctypes.c_double), ("Hz", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("T_start", ctypes.c_double), ("T_end", ctypes.c_double), ("cool", ctypes.c_double),
                ("sweeps_per_T", ctypes.c_int64), ("sweeps_final", ctypes.c_int64),
                ("cone0", ctypes.c_double), ("acc_target", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("segment_pairs", ctypes.c_int32)]


SCHED_DEFAULT, SCHED_ONE_PASS, SCHED_TWO_PASS, SCHED_LAG_SPLIT, SCHED_FOLD = 0, 1, 2, 3, 4
SCHEDULES = {"default": SCHED_DEFAULT, "one_pass": SCHED_ONE_PASS, "two_pass": SCHED_TWO_PASS,
             "lag_split": SCHED_LAG_SPLIT, "fold": SCHED_FOLD}


class SqSpec(ctypes.Structure):
    _fields_ = [("n_origins", ctypes.c_int32), ("n_lags", ctypes.c_int32),
                ("origin_stride", ctypes.c_int32), ("flags", ctypes.c_int32)]


class TrajSpec(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("cells", ctypes.c_int32 * 3),
                ("coupling", ctypes.c_int32), ("r_cut", ctypes.c_float), ("J", ctypes.c_double),
                ("dt", ctypes.c_double), ("init", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("sigma", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("init_dev", ctypes.c_void_p), ("D", ctypes.c_double), ("A", ctypes.c_double),
                ("Hz", ctypes.c_double)]


EXPORTS = ("sdc_plan_create", "sdc_plan_n_bins", "sdc_accumulate", "sdc_finalize", "sdc_plan_raw",
           "sdc_plan_load_raw", "sdc_plan_timings", "sdc_plan_reset", "sdc_plan_destroy",
           "sdc_status_string", "sdc_last_error", "sdc_layout_keys", "sdc_traj_generate",
           "sdc_batch_create", "sdc_batch_accumulate", "sdc_batch_timings", "sdc_batch_info",
           "sdc_batch_destroy", "sdc_plan_structure_factor", "sdc_sq_create", "sdc_sq_accumulate",
           "sdc_sq_finalize", "sdc_sq_timings", "sdc_sq_reset", "sdc_sq_destroy", "sdc_mc_n_sweeps",
           "sdc_mc_anneal", "sdc_mc_create", "sdc_mc_run", "sdc_mc_timings", "sdc_mc_uses_stencil",
           "sdc_mc_destroy", "sdc_plan_create_tuned", "sdc_plan_get_tuning", "sdc_autotune",
           "sdc_tuning_lookup", "sdc_batch_create_tuned", "sdc_batch_schedule",
           "sdc_plan_structure_factor_static", "sdc_mfma_peak", "sdc_mfma_probe",
           "sdc_autotune_candidates")
MFMA_FORMS = {"bf16": 0, "f16": 1, "f32": 2}
FLAG_TIMING = 1
FLAG_CONNECTED = 2
FLAG_NO_KEY_TABLE = 4
FLAG_DETERMINISTIC = 8

_lib = None


def lib():
    """Load libsdc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2308_07487_amd.build` (no fallback path exists)")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.sdc_plan_create.argtypes = [P, i64, ctypes.POINTER(BinSpec), ctypes.POINTER(CorrSpec),
                                      ctypes.c_int, ctypes.POINTER(P)]
        L.sdc_plan_n_bins.argtypes = [P, ctypes.POINTER(i64)]
        L.sdc_plan_create_tuned.argtypes = [P, i64, ctypes.POINTER(BinSpec), ctypes.POINTER(CorrSpec),
                                            ctypes.POINTER(Tuning), ctypes.c_int, ctypes.POINTER(P)]
        L.sdc_plan_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        L.sdc_autotune.argtypes = [P, i64, ctypes.POINTER(BinSpec), ctypes.POINTER(CorrSpec), ctypes.c_int,
                                   i32, P, i32, ctypes.c_char_p, ctypes.POINTER(Tuning),
                                   ctypes.POINTER(ctypes.c_double), P]
        L.sdc_autotune_candidates.argtypes = [ctypes.POINTER(BinSpec), ctypes.POINTER(CorrSpec), P, i32,
                                              ctypes.POINTER(i32)]
        L.sdc_tuning_lookup.argtypes = [ctypes.c_char_p, i64, ctypes.POINTER(BinSpec), ctypes.POINTER(CorrSpec),
                                        ctypes.c_int, ctypes.POINTER(Tuning), ctypes.POINTER(i32)]
        L.sdc_batch_create_tuned.argtypes = [P, i32, i32, ctypes.POINTER(Tuning), ctypes.POINTER(P)]
        L.sdc_batch_schedule.argtypes = [P, ctypes.POINTER(i32)]
        L.sdc_accumulate.argtypes = [P, P, i64, P, i32, P]
        L.sdc_finalize.argtypes = [P, P, P, P, P, P, P, P]
        L.sdc_plan_raw.argtypes = [P, P, P, P, P, P]
        L.sdc_plan_load_raw.argtypes = [P, P, P, P, P, P]
        L.sdc_plan_timings.argtypes = [P, P]
        L.sdc_plan_reset.argtypes = [P, P]
        L.sdc_plan_destroy.argtypes = [P]
        L.sdc_status_string.argtypes = [ctypes.c_int]
        L.sdc_status_string.restype = ctypes.c_char_p
        L.sdc_last_error.argtypes = []
        L.sdc_last_error.restype = ctypes.c_char_p
        L.sdc_layout_keys.argtypes = [P, i64, ctypes.POINTER(BinSpec), P]
        L.sdc_traj_generate.argtypes = [P, i64, ctypes.POINTER(TrajSpec), P, i64, ctypes.c_int, P]
        L.sdc_batch_create.argtypes = [P, i32, i32, ctypes.POINTER(P)]
        L.sdc_batch_timings.argtypes = [P, P]
        L.sdc_batch_accumulate.argtypes = [P, P, P, P]
        L.sdc_batch_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i32)]
        L.sdc_batch_destroy.argtypes = [P]
        L.sdc_plan_structure_factor.argtypes = [P, P, i32, P, P, P]
        L.sdc_plan_structure_factor_static.argtypes = [P, P, i32, P, P, P]
        L.sdc_mfma_peak.argtypes = [i32, i32, i64, i32, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
        L.sdc_mfma_probe.argtypes = [i32, ctypes.c_float, P, P, i32, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]
        L.sdc_mc_n_sweeps.argtypes = [ctypes.POINTER(McSpec), ctypes.POINTER(i64)]
        L.sdc_mc_anneal.argtypes = [P, i64, ctypes.POINTER(McSpec), P, P, P, P, ctypes.c_int, P]
        L.sdc_mc_create.argtypes = [P, i64, ctypes.POINTER(McSpec), ctypes.c_int, ctypes.POINTER(P)]
        L.sdc_mc_run.argtypes = [P, ctypes.POINTER(McSpec), P, P, P, P, P]
        L.sdc_mc_timings.argtypes = [P, P]
        L.sdc_mc_uses_stencil.argtypes = [P, ctypes.POINTER(i32)]
        L.sdc_mc_destroy.argtypes = [P]
        L.sdc_sq_create.argtypes = [P, i64, P, i32, ctypes.POINTER(SqSpec), ctypes.c_int, ctypes.POINTER(P)]
        L.sdc_sq_accumulate.argtypes = [P, P, i64, P]
        L.sdc_sq_finalize.argtypes = [P, P, P, P]
        L.sdc_sq_timings.argtypes = [P, P]
        L.sdc_sq_reset.argtypes = [P, P]
        L.sdc_sq_destroy.argtypes = [P]
        for name in EXPORTS:
            if name not in ("sdc_status_string", "sdc_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(s):
    return lib().sdc_status_string(int(s)).decode()


def last_error():
    return lib().sdc_last_error().decode()


def _check(status, what):
    if status != OK:
        raise SdcError(status, what, last_error())


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype_name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if str(t.dtype) != dtype_name or not t.is_contiguous():
        raise TypeError(f"expected a contiguous {dtype_name} tensor")
    return ctypes.c_void_p(t.data_ptr())


def bin_spec(kind, cells=(0, 0, 0), n_shells=0, r_max=0.0):
    b = BinSpec()
    b.kind = int(kind)
    for a in range(3):
        b.cells[a] = int(cells[a])
    b.n_shells = int(n_shells)
    b.r_max = float(r_max)
    return b


def corr_spec(n_origins, n_lags, precision="split_bf16", origin_stride=1, flags=0):
    c = CorrSpec()
    c.n_origins = int(n_origins)
    c.n_lags = int(n_lags)
    c.origin_stride = int(origin_stride)
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c.flags = int(flags)
    return c


def tuning(schedule=None, segment_pairs=None):
    """Tuning struct from a schedule name or code and a segment length (None = default)."""
    sch = SCHEDULES.get(schedule, schedule) if schedule is not None else SCHED_DEFAULT
    return Tuning(int(sch), int(segment_pairs or 0))


def _tuning_dict(t):
    inv = {v: k for k, v in SCHEDULES.items()}
    return {"schedule": inv.get(t.schedule, t.schedule), "segment_pairs": int(t.segment_pairs)}


def autotune(positions, kind, n_origins, n_lags, precision="split_bf16", cells=(0, 0, 0), n_shells=0,
             r_max=0.0, origin_stride=1, connected=False, device=0, max_lags=0, candidates=None, cache_path=None):
    """Times candidate tunings of this sample shape on the device
    (sdc_autotune).  candidates: list of (schedule, segment_pairs), or None for
    the built-in list.  Returns (best {"schedule", "segment_pairs"}, its
    median fused ms, [(candidate dict, median ms), ...]).  With cache_path the
    winner is written to that JSON tuning file."""
    pos = np.ascontiguousarray(positions, dtype=np.float32)
    bs = bin_spec(kind, cells, n_shells, r_max)
    cs = corr_spec(n_origins, n_lags, precision, origin_stride, flags=FLAG_CONNECTED if connected else 0)
    if candidates is None:
        n = ctypes.c_int32()
        _check(lib().sdc_autotune_candidates(ctypes.byref(bs), ctypes.byref(cs), None, 0, ctypes.byref(n)),
               "sdc_autotune_candidates")
        arr = (Tuning * n.value)()
        _check(lib().sdc_autotune_candidates(ctypes.byref(bs), ctypes.byref(cs), ctypes.cast(arr, ctypes.c_void_p),
                                             n.value, ctypes.byref(n)), "sdc_autotune_candidates")
    else:
        arr = (Tuning * len(candidates))(*[tuning(sch, seg) for sch, seg in candidates])
    times = np.zeros(len(arr))
    best = Tuning()
    ms = ctypes.c_double()
    _check(lib().sdc_autotune(_np_ptr(pos), pos.shape[0], ctypes.byref(bs), ctypes.byref(cs), int(device),
                              int(max_lags), ctypes.cast(arr, ctypes.c_void_p), len(arr),
                              cache_path.encode() if cache_path else None, ctypes.byref(best), ctypes.byref(ms),
                              _np_ptr(times)), "sdc_autotune")
    return _tuning_dict(best), float(ms.value), [(_tuning_dict(t), float(x)) for t, x in zip(arr, times)]


def tuning_lookup(cache_path, n_sites, kind, n_origins, n_lags, precision="split_bf16", cells=(0, 0, 0),
                  n_shells=0, r_max=0.0, device=0):
    """The tuning-file entry of a sample shape, or None."""
    bs = bin_spec(kind, cells, n_shells, r_max)
    cs = corr_spec(n_origins, n_lags, precision)
    t = Tuning()
    found = ctypes.c_int32()
    _check(lib().sdc_tuning_lookup(cache_path.encode(), int(n_sites), ctypes.byref(bs), ctypes.byref(cs),
                                   int(device), ctypes.byref(t), ctypes.byref(found)), "sdc_tuning_lookup")
    return _tuning_dict(t) if found.value else None


def mfma_peak(form="bf16", random_operands=True, iterations=20000, workgroups_per_cu=2, device=0):
    """Sustained MFMA rate (sdc_mfma_peak): (ms of the timed launch, executed TFLOP/s)."""
    ms, tf = ctypes.c_double(), ctypes.c_double()
    _check(lib().sdc_mfma_peak(MFMA_FORMS[form], int(bool(random_operands)), int(iterations),
                               int(workgroups_per_cu), int(device), ctypes.byref(ms), ctypes.byref(tf)),
           "sdc_mfma_peak")
    return float(ms.value), float(tf.value)


def mfma_probe(form, c, a, b, device=0):
    """c + sum_k a[k] b[k] through one MFMA instruction of the form (sdc_mfma_probe)."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    out = ctypes.c_float()
    _check(lib().sdc_mfma_probe(MFMA_FORMS[form], float(c), _np_ptr(a), _np_ptr(b), a.shape[0], int(device),
                                ctypes.byref(out)), "sdc_mfma_probe")
    return float(out.value)


def layout_keys(positions, kind, cells=(0, 0, 0), n_shells=0, r_max=0.0):
    """Host check of the tile layout: bin of every ordered pair [n][n]."""
    pos = np.ascontiguousarray(positions, dtype=np.float32)
    n = pos.shape[0]
    out = np.zeros((n, n), dtype=np.int64)
    b = bin_spec(kind, cells, n_shells, r_max)
    _check(lib().sdc_layout_keys(_np_ptr(pos), n, ctypes.byref(b), _np_ptr(out)), "sdc_layout_keys")
    return out


class Plan:
    """One sample's plan: positions and bin spec fixed, accumulation state on the GPU."""

    def __init__(self, positions, kind, n_origins, n_lags, precision="split_bf16", cells=(0, 0, 0),
                 n_shells=0, r_max=0.0, origin_stride=1, device=0, timing=False, connected=False,
                 key_table=True, deterministic=False, schedule=None, segment_pairs=None):
        self._h = None
        pos = np.ascontiguousarray(positions, dtype=np.float32)
        self.n_sites = pos.shape[0]
        self.n_origins = int(n_origins)
        self.n_lags = int(n_lags)
        self.origin_stride = int(origin_stride)
        self.bins = bin_spec(kind, cells, n_shells, r_max)
        self.corr = corr_spec(n_origins, n_lags, precision, origin_stride,
                              flags=(FLAG_TIMING if timing else 0) | (FLAG_CONNECTED if connected else 0)
                              | (0 if key_table else FLAG_NO_KEY_TABLE)
                              | (FLAG_DETERMINISTIC if deterministic else 0))
        self.device = int(device)
        h = ctypes.c_void_p()
        if schedule is None and segment_pairs is None:
            _check(lib().sdc_plan_create(_np_ptr(pos), self.n_sites, ctypes.byref(self.bins),
                                         ctypes.byref(self.corr), self.device, ctypes.byref(h)),
                   "sdc_plan_create")
        else:
            tu = tuning(schedule, segment_pairs)
            _check(lib().sdc_plan_create_tuned(_np_ptr(pos), self.n_sites, ctypes.byref(self.bins),
                                               ctypes.byref(self.corr), ctypes.byref(tu), self.device,
                                               ctypes.byref(h)), "sdc_plan_create_tuned")
        self._h = h
        nb = ctypes.c_int64()
        _check(lib().sdc_plan_n_bins(self._h, ctypes.byref(nb)), "sdc_plan_n_bins")
        self.n_bins = int(nb.value)

    @property
    def tuning(self):
        """{"schedule", "segment_pairs"} the plan runs with."""
        t = Tuning()
        _check(lib().sdc_plan_get_tuning(self._h, ctypes.byref(t)), "sdc_plan_get_tuning")
        return _tuning_dict(t)

    def accumulate(self, spins, lags=None, stream=None):
        """spins: contiguous float32 device tensor [T][N][3]."""
        if tuple(spins.shape[1:]) != (self.n_sites, 3):
            raise ValueError("spins must have shape [T][n_sites][3]")
        ptr = _dev_ptr(spins, "torch.float32")
        if lags is None:
            lp, nl = None, 0
        else:
            la = np.ascontiguousarray(lags, dtype=np.int32)
            lp, nl = _np_ptr(la), la.shape[0]
        _check(lib().sdc_accumulate(self._h, ptr, spins.shape[0], lp, nl, _stream_ptr(stream)),
               "sdc_accumulate")

    def finalize(self, stream=None, want_C=True):
        """Returns dict with C [n_lags][n_bins], counts, Csum, Cself, Ssum, Sself (complex)."""
        nl, nb = self.n_lags, self.n_bins
        C = np.zeros((nl, nb), dtype=np.float64) if want_C else None
        counts = np.zeros(nb, dtype=np.uint64)
        cs = np.zeros(nl)
        cf = np.zeros(nl)
        ss = np.zeros((nl, 2))
        sf = np.zeros((nl, 2))
        _check(lib().sdc_finalize(self._h, _np_ptr(C) if C is not None else None, _np_ptr(counts),
                                  _np_ptr(cs), _np_ptr(cf), _np_ptr(ss), _np_ptr(sf),
                                  _stream_ptr(stream)), "sdc_finalize")
        return dict(C=C, counts=counts, Csum=cs, Cself=cf, Ssum=ss[:, 0] + 1j * ss[:, 1],
                    Sself=sf[:, 0] + 1j * sf[:, 1])

    def raw(self, stream=None):
        """(H [n_lags][n_bins], n_org [n_lags], self [n_lags], msum [n_lags]) as
        accumulated (FP64); msum = sum over origins of M(o s).M(o s + t)."""
        H = np.zeros((self.n_lags, self.n_bins))
        no = np.zeros(self.n_lags)
        sf = np.zeros(self.n_lags)
        ms = np.zeros(self.n_lags)
        _check(lib().sdc_plan_raw(self._h, _np_ptr(H), _np_ptr(no), _np_ptr(sf), _np_ptr(ms),
                                  _stream_ptr(stream)), "sdc_plan_raw")
        return H, no, sf, ms

    def load_raw(self, H, n_org, self_raw, msum, stream=None):
        H = np.ascontiguousarray(H, dtype=np.float64)
        n_org = np.ascontiguousarray(n_org, dtype=np.float64)
        self_raw = np.ascontiguousarray(self_raw, dtype=np.float64)
        msum = np.ascontiguousarray(msum, dtype=np.float64)
        _check(lib().sdc_plan_load_raw(self._h, _np_ptr(H), _np_ptr(n_org), _np_ptr(self_raw), _np_ptr(msum),
                                       _stream_ptr(stream)), "sdc_plan_load_raw")

    def structure_factor(self, m, stream=None):
        """S(q, t) and its windowed transform for q_a = 2 pi m_a / L_a (periodic
        plans): returns (Sqt [n_q][n_lags], Sqw [n_q][n_lags]), complex128."""
        m = np.ascontiguousarray(np.atleast_2d(m), dtype=np.int32)
        if m.shape[1] != 3:
            raise ValueError("m must have shape [n_q][3]")
        sqt = np.zeros((m.shape[0], self.n_lags, 2))
        sqw = np.zeros((m.shape[0], self.n_lags, 2))
        _check(lib().sdc_plan_structure_factor(self._h, _np_ptr(m), m.shape[0], _np_ptr(sqt), _np_ptr(sqw),
                                               _stream_ptr(stream)), "sdc_plan_structure_factor")
        return sqt[..., 0] + 1j * sqt[..., 1], sqw[..., 0] + 1j * sqw[..., 1]

    def structure_factor_static(self, m, stream=None):
        """structure_factor through sdc_plan_structure_factor_static (fixed
        device scratch, no allocation; n_q * n_lags limited)."""
        m = np.ascontiguousarray(np.atleast_2d(m), dtype=np.int32)
        if m.shape[1] != 3:
            raise ValueError("m must have shape [n_q][3]")
        sqt = np.zeros((m.shape[0], self.n_lags, 2))
        sqw = np.zeros((m.shape[0], self.n_lags, 2))
        _check(lib().sdc_plan_structure_factor_static(self._h, _np_ptr(m), m.shape[0], _np_ptr(sqt),
                                                      _np_ptr(sqw), _stream_ptr(stream)),
               "sdc_plan_structure_factor_static")
        return sqt[..., 0] + 1j * sqt[..., 1], sqw[..., 0] + 1j * sqw[..., 1]

    def timings(self):
        """(pack_ms, self_ms, fused_ms) of the last accumulate (timing plans only)."""
        ms = np.zeros(3)
        _check(lib().sdc_plan_timings(self._h, _np_ptr(ms)), "sdc_plan_timings")
        return tuple(float(x) for x in ms)

    def reset(self, stream=None):
        _check(lib().sdc_plan_reset(self._h, _stream_ptr(stream)), "sdc_plan_reset")

    def close(self):
        if self._h is not None:
            _check(lib().sdc_plan_destroy(self._h), "sdc_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Several plans accumulated with one persistent fused launch (all lags)."""

    def __init__(self, plans, timing=False, schedule=None):
        self._h = None
        self.plans = list(plans)  # keeps the plans alive while the batch exists
        arr = (ctypes.c_void_p * len(self.plans))(*[p._h.value for p in self.plans])
        h = ctypes.c_void_p()
        if schedule is None:
            _check(lib().sdc_batch_create(ctypes.cast(arr, ctypes.c_void_p), len(self.plans),
                                          FLAG_TIMING if timing else 0, ctypes.byref(h)), "sdc_batch_create")
        else:
            tu = tuning(schedule)
            _check(lib().sdc_batch_create_tuned(ctypes.cast(arr, ctypes.c_void_p), len(self.plans),
                                                FLAG_TIMING if timing else 0, ctypes.byref(tu), ctypes.byref(h)),
                   "sdc_batch_create_tuned")
        self._h = h

    @property
    def schedule(self):
        """Schedule name of the batch's launch."""
        v = ctypes.c_int32()
        _check(lib().sdc_batch_schedule(self._h, ctypes.byref(v)), "sdc_batch_schedule")
        return {v_: k for k, v_ in SCHEDULES.items()}.get(v.value, v.value)

    def timings(self):
        """(pack_and_self_ms, fused_ms) of the last accumulate (timing batches only)."""
        ms = np.zeros(2)
        _check(lib().sdc_batch_timings(self._h, _np_ptr(ms)), "sdc_batch_timings")
        return float(ms[0]), float(ms[1])

    def accumulate(self, spins_list, stream=None):
        """spins_list[k]: contiguous float32 device tensor [T_k][N_k][3] for plan k."""
        if len(spins_list) != len(self.plans):
            raise ValueError("one trajectory per plan")
        for p, sp in zip(self.plans, spins_list):
            if tuple(sp.shape[1:]) != (p.n_sites, 3):
                raise ValueError("spins must have shape [T][n_sites][3]")
        ptrs = (ctypes.c_void_p * len(spins_list))(*[_dev_ptr(sp, "torch.float32").value for sp in spins_list])
        nf = np.ascontiguousarray([sp.shape[0] for sp in spins_list], dtype=np.int64)
        _check(lib().sdc_batch_accumulate(self._h, ctypes.cast(ptrs, ctypes.c_void_p), _np_ptr(nf),
                                          _stream_ptr(stream)), "sdc_batch_accumulate")

    def info(self):
        """(total fused tasks, persistent grid size)."""
        nt, g = ctypes.c_int64(), ctypes.c_int32()
        _check(lib().sdc_batch_info(self._h, ctypes.byref(nt), ctypes.byref(g)), "sdc_batch_info")
        return int(nt.value), int(g.value)

    def close(self):
        if self._h is not None:
            _check(lib().sdc_batch_destroy(self._h), "sdc_batch_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def traj_generate(positions, kind, frames_out, cells=(0, 0, 0), J=1.0, dt=0.01, coupling=0,
                  r_cut=0.0, init=INIT_UNIFORM, sigma=0.0, seed=0, init_state=None, device=0,
                  stream=None, D=0.0, A=0.0, Hz=0.0):
    """LL RK4 frames into frames_out (float32 device tensor [T][N][3]); D, A, Hz:
    the DMI, anisotropy and field terms of Eq. (1)."""
    pos = np.ascontiguousarray(positions, dtype=np.float32)
    sp = TrajSpec()
    sp.kind = int(kind)
    for a in range(3):
        sp.cells[a] = int(cells[a])
    sp.coupling = int(coupling)
    sp.r_cut = float(r_cut)
    sp.J = float(J)
    sp.dt = float(dt)
    sp.init = int(init)
    sp.sigma = float(sigma)
    sp.seed = int(seed)
    sp.init_dev = _dev_ptr(init_state, "torch.float32").value if init_state is not None else None
    sp.D, sp.A, sp.Hz = float(D), float(A), float(Hz)
    if tuple(frames_out.shape[1:]) != (pos.shape[0], 3):
        raise ValueError("frames_out must have shape [T][n_sites][3]")
    _check(lib().sdc_traj_generate(_np_ptr(pos), pos.shape[0], ctypes.byref(sp),
                                   _dev_ptr(frames_out, "torch.float32"), frames_out.shape[0],
                                   int(device), _stream_ptr(stream)), "sdc_traj_generate")


def mc_spec(kind, cells=(0, 0, 0), coupling=COUPLING_NN_UNIFORM, r_cut=0.0, J=1.0, D=0.0, A=0.0, Hz=0.0,
            seed=0, T_start=1.0, T_end=1.0, cool=0.9, sweeps_per_T=1, sweeps_final=0, cone0=np.pi,
            acc_target=0.2):
    m = McSpec()
    m.kind = int(kind)
    for a in range(3):
        m.cells[a] = int(cells[a])
    m.coupling, m.r_cut = int(coupling), float(r_cut)
    m.J, m.D, m.A, m.Hz = float(J), float(D), float(A), float(Hz)
    m.seed = int(seed)
    m.T_start, m.T_end, m.cool = float(T_start), float(T_end), float(cool)
    m.sweeps_per_T, m.sweeps_final = int(sweeps_per_T), int(sweeps_final)
    m.cone0, m.acc_target = float(cone0), float(acc_target)
    return m


def mc_n_sweeps(spec):
    n = ctypes.c_int64()
    _check(lib().sdc_mc_n_sweeps(ctypes.byref(spec), ctypes.byref(n)), "sdc_mc_n_sweeps")
    return int(n.value)


def mc_anneal(positions, spec, init_state, state_out, device=0, stream=None, history=True):
    """Annealed Metropolis sweeps (Sec. 2.1, Sec. 4.3) from init_state into
    state_out (float32 device tensors [N][3]).  Returns (accepted moves per
    sweep or None, energy per site, final cone, last T, colour classes)."""
    pos = np.ascontiguousarray(positions, dtype=np.float32)
    n = pos.shape[0]
    for t in (init_state, state_out):
        if tuple(t.shape) != (n, 3):
            raise ValueError("states must have shape [n_sites][3]")
    acc = np.zeros(max(mc_n_sweeps(spec), 1), dtype=np.int64) if history else None
    info = np.zeros(4)
    _check(lib().sdc_mc_anneal(_np_ptr(pos), n, ctypes.byref(spec), _dev_ptr(init_state, "torch.float32"),
                               _dev_ptr(state_out, "torch.float32"), _np_ptr(acc) if history else None,
                               _np_ptr(info), int(device), _stream_ptr(stream)), "sdc_mc_anneal")
    if history:
        acc = acc[:mc_n_sweeps(spec)]
    return acc, float(info[0]), float(info[1]), float(info[2]), int(info[3])


class MonteCarlo:
    """Reusable annealed Metropolis sweeps on one sample (bonds and colour
    classes built once)."""

    def __init__(self, positions, spec, device=0):
        self._h = None
        pos = np.ascontiguousarray(positions, dtype=np.float32)
        self.n_sites = pos.shape[0]
        h = ctypes.c_void_p()
        _check(lib().sdc_mc_create(_np_ptr(pos), self.n_sites, ctypes.byref(spec), int(device), ctypes.byref(h)),
               "sdc_mc_create")
        self._h = h

    def run(self, schedule, state_out, init_state=None, stream=None, history=False, info=False):
        """Run schedule's sweeps (from init_state, or from the previous run's
        state); returns (accepted per sweep or None, info array or None)."""
        if tuple(state_out.shape) != (self.n_sites, 3):
            raise ValueError("states must have shape [n_sites][3]")
        acc = np.zeros(max(mc_n_sweeps(schedule), 1), dtype=np.int64) if history else None
        inf = np.zeros(4) if info else None
        ip = _dev_ptr(init_state, "torch.float32") if init_state is not None else None
        _check(lib().sdc_mc_run(self._h, ctypes.byref(schedule), ip, _dev_ptr(state_out, "torch.float32"),
                                _np_ptr(acc) if history else None, _np_ptr(inf) if info else None,
                                _stream_ptr(stream)), "sdc_mc_run")
        return (acc[:mc_n_sweeps(schedule)] if history else None), inf

    def timings(self):
        ms = np.zeros(1)
        _check(lib().sdc_mc_timings(self._h, _np_ptr(ms)), "sdc_mc_timings")
        return float(ms[0])

    @property
    def uses_stencil(self):
        """True when the sweeps compute neighbours by lattice arithmetic
        instead of reading the bond tables (same results)."""
        v = ctypes.c_int32()
        _check(lib().sdc_mc_uses_stencil(self._h, ctypes.byref(v)), "sdc_mc_uses_stencil")
        return bool(v.value)

    def close(self):
        if self._h is not None:
            _check(lib().sdc_mc_destroy(self._h), "sdc_mc_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class StructureFactor:
    """Eq. (3) at arbitrary wave vectors for any point set, accumulated on the GPU."""

    def __init__(self, positions, q, n_origins, n_lags, origin_stride=1, device=0, timing=False,
                 connected=False):
        self._h = None
        pos = np.ascontiguousarray(positions, dtype=np.float32)
        qv = np.ascontiguousarray(np.atleast_2d(q), dtype=np.float64)
        if pos.ndim != 2 or pos.shape[1] != 3 or qv.shape[1] != 3:
            raise ValueError("positions and q must have shape [n][3]")
        self.n_sites, self.n_q = pos.shape[0], qv.shape[0]
        self.n_lags = int(n_lags)
        self.spec = SqSpec(int(n_origins), int(n_lags), int(origin_stride),
                           (FLAG_TIMING if timing else 0) | (FLAG_CONNECTED if connected else 0))
        h = ctypes.c_void_p()
        _check(lib().sdc_sq_create(_np_ptr(pos), self.n_sites, _np_ptr(qv), self.n_q, ctypes.byref(self.spec),
                                   int(device), ctypes.byref(h)), "sdc_sq_create")
        self._h = h

    def accumulate(self, spins, stream=None):
        """spins: contiguous float32 device tensor [T][N][3]."""
        if tuple(spins.shape[1:]) != (self.n_sites, 3):
            raise ValueError("spins must have shape [T][n_sites][3]")
        _check(lib().sdc_sq_accumulate(self._h, _dev_ptr(spins, "torch.float32"), spins.shape[0],
                                       _stream_ptr(stream)), "sdc_sq_accumulate")

    def finalize(self, stream=None):
        """(Sqt [n_q][n_lags], Sqw [n_q][n_lags]) complex128."""
        sqt = np.zeros((self.n_q, self.n_lags, 2))
        sqw = np.zeros((self.n_q, self.n_lags, 2))
        _check(lib().sdc_sq_finalize(self._h, _np_ptr(sqt), _np_ptr(sqw), _stream_ptr(stream)), "sdc_sq_finalize")
        return sqt[..., 0] + 1j * sqt[..., 1], sqw[..., 0] + 1j * sqw[..., 1]

    def timings(self):
        """(pack_ms, contraction_ms, reduce_and_correlation_ms) of the last accumulate
        (timing accumulators only)."""
        ms = np.zeros(3)
        _check(lib().sdc_sq_timings(self._h, _np_ptr(ms)), "sdc_sq_timings")
        return float(ms[0]), float(ms[1]), float(ms[2])

    def reset(self, stream=None):
        _check(lib().sdc_sq_reset(self._h, _stream_ptr(stream)), "sdc_sq_reset")

    def close(self):
        if self._h is not None:
            _check(lib().sdc_sq_destroy(self._h), "sdc_sq_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

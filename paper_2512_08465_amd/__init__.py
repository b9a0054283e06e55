"""MI355X contingency screening: Python binding of the C-ABI in include/cs.h.

Argument marshalling only; every step of the screening runs in the HIP
library ``libcs.so`` built in this directory.  Importing works without a GPU;
creating a context requires one and fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes
import os
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcs.so")

CS_OK, CS_EINVAL, CS_ENOMEM, CS_EHBM, CS_EDEVICE, CS_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
CS_EAGAIN, CS_ETIMEDOUT = -6, -7
PREC_FP64, PREC_MIXED = 0, 1
# launch variants of the large-order LU, in the autotuner's order: panel
# widths 16, 32, 64 (right-looking), panels of 16 / 32 in groups of 64
TUNE_VARIANTS = (16, 32, 64, 1664, 3264)   # large-order LU (order > REG_ORDER)
REG_TUNE_VARIANTS = (4, 8)                  # wavefronts per matrix (order <= REG_ORDER)
REG_ORDER, REG_ORDER_W4 = 1024, 768
CAUSE_ISLAND, CAUSE_OPF, CAUSE_LIMIT, CAUSE_SSS, CAUSE_NUMERICAL = 1, 2, 4, 8, 16
CAUSE_PRUNED = 32
OPF_CONVERGED, OPF_MAXIT, OPF_NUMERICAL, OPF_NOT_RUN = 0, 1, 2, 3
NEAR_SSS, NEAR_OPF, NEAR_LIMIT = 1, 2, 4
N_DYN = 14

RESULT_DTYPE = np.dtype([
    ("severe", np.uint8), ("cause", np.uint8), ("opf_status", np.uint8), ("near", np.uint8),
    ("n_islands", np.int16), ("opf_iters", np.int16), ("n_states", np.int32),
    ("reserved", np.int32), ("opf_cost", np.float64), ("max_real_eig", np.float64),
    ("min_damping", np.float64), ("max_violation", np.float64)])
assert RESULT_DTYPE.itemsize == 48


class CSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"cs error {code}: {msg}")
        self.code = code


class _NetDesc(ctypes.Structure):
    _fields_ = [("n_bus", ctypes.c_int32), ("n_branch", ctypes.c_int32),
                ("n_gen", ctypes.c_int32), ("n_load", ctypes.c_int32),
                ("ref_bus", ctypes.c_int32), ("base_mva", ctypes.c_double),
                ("f_hz", ctypes.c_double)] + \
               [(k, ctypes.c_void_p) for k in (
                   "vmin", "vmax", "gs", "bs", "br_from", "br_to", "br_r", "br_x",
                   "br_b", "br_rate", "br_tap", "br_shift", "gen_bus", "gen_kind",
                   "pmin", "pmax", "qmin", "qmax", "c2", "c1", "c0", "dyn",
                   "load_bus", "pd", "qd")]


class RiskOptions(ctypes.Structure):
    _fields_ = [("severity", ctypes.c_int32), ("zeta_ref", ctypes.c_double),
                ("n_cc", ctypes.c_int64), ("cc_pairs", ctypes.c_void_p),
                ("cc_rate", ctypes.c_void_p)]


SEV_BINARY, SEV_DAMPING = 0, 1


class Options(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("max_it", ctypes.c_int32),
                ("tol", ctypes.c_double), ("near_eps", ctypes.c_double),
                ("hbm_budget", ctypes.c_size_t), ("batch", ctypes.c_int32),
                ("timing", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("refine_steps", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("autotune", ctypes.c_int32)]


KERNELS = ("topology", "kkt_assemble", "kkt_lu", "ipm_update", "dyn_assemble", "dyn_lu",
           "state_matrix", "eig", "classify", "risk", "kkt_refine", "kkt_lu64")


class Stats(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(KERNELS)),
                ("launches", ctypes.c_int64 * len(KERNELS)),
                ("units", ctypes.c_int64 * len(KERNELS)),
                ("kkt_order", ctypes.c_int64), ("dyn_order", ctypes.c_int64)]


_lib = None


def library():
    """Load libcs.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2512_08465_amd.build`")
    # PyTorch provides device memory and streams, so the process must use its
    # HIP runtime: load it first, and libcs.so binds to the same
    # libamdhip64.so.7 instead of loading a second runtime.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    sig = {
        "cs_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(vp)]),
        "cs_ctx_destroy": (None, [vp]),
        "cs_net_create": (ctypes.c_int, [vp, ctypes.POINTER(_NetDesc), ctypes.POINTER(vp)]),
        "cs_net_destroy": (None, [vp]),
        "cs_opts_default": (None, [ctypes.POINTER(Options)]),
        "cs_screen": (ctypes.c_int, [vp, vp, vp, i64, dp, ctypes.POINTER(Options), vp, dp]),
        "cs_screen_device": (ctypes.c_int, [vp, vp, vp, i64, dp, ctypes.POINTER(Options),
                                            vp, dp, vp]),
        "cs_detail": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(Options), vp, dp, dp, dp,
                                     dp, dp, dp, vp, vp]),
        "cs_dense_solve_batched": (ctypes.c_int, [vp, dp, i32, i32, i32, i32, vp, vp]),
        "cs_eigvals_batched": (ctypes.c_int, [vp, dp, i32, i32, i32, dp, dp, vp, vp]),
        "cs_kkt_at": (ctypes.c_int, [vp, vp, vp, i32, dp, dp, dp, dp, dp, dp, vp, vp]),
        "cs_screen_detail": (ctypes.c_int, [vp, vp, vp, i64, ctypes.POINTER(Options), vp,
                                            dp, dp, dp, dp, dp, dp, vp]),
        "cs_dyn_at": (ctypes.c_int, [vp, vp, vp, dp, dp, dp, dp, dp, vp, dp, dp]),
        "cs_screen_device_noalloc": (ctypes.c_int, [vp, vp, vp, i64, dp,
                                                    ctypes.POINTER(Options), vp, dp, vp]),
        "cs_risk_opts_default": (None, [ctypes.POINTER(RiskOptions)]),
        "cs_screen3_device": (ctypes.c_int, [vp, vp, vp, i64, dp, ctypes.POINTER(Options),
                                             vp, dp, vp]),
        "cs_screen_n3_device": (ctypes.c_int, [vp, vp, vp, i64, vp, i64, vp, dp,
                                               ctypes.POINTER(Options), vp, dp,
                                               ctypes.POINTER(ctypes.c_int64), vp]),
        "cs_risk": (ctypes.c_int, [vp, vp, vp, i64, vp, dp, ctypes.POINTER(RiskOptions), dp,
                                   vp]),
        "cs_risk_mc": (ctypes.c_int, [vp, vp, vp, i64, vp, dp, i64, ctypes.POINTER(RiskOptions),
                                      dp, dp, vp, vp]),
        "cs_stats_get": (ctypes.c_int, [vp, ctypes.POINTER(Stats)]),
        "cs_stats_reset": (ctypes.c_int, [vp]),
        "cs_last_error": (ctypes.c_char_p, []),
        "cs_abi_version": (ctypes.c_int, []),
        "cs_server_create": (ctypes.c_int, [vp, vp, ctypes.POINTER(Options), i64,
                                            ctypes.POINTER(vp)]),
        "cs_server_destroy": (None, [vp]),
        "cs_submit": (ctypes.c_int, [vp, vp, i64, dp, ctypes.POINTER(vp)]),
        "cs_submit_snapshot": (ctypes.c_int, [vp, vp, i64, dp, dp, ctypes.POINTER(vp)]),
        "cs_server_create_multi": (ctypes.c_int, [vp, ctypes.POINTER(vp), ctypes.c_int, dp,
                                                  ctypes.POINTER(Options), i64,
                                                  ctypes.POINTER(vp)]),
        "cs_server_slots": (ctypes.c_int, [vp, ctypes.c_int]),
        "cs_submit_net": (ctypes.c_int, [vp, ctypes.c_int, vp, i64, dp, dp, ctypes.POINTER(vp)]),
        "cs_autotune": (ctypes.c_int, [vp, i32, i32, i32, ctypes.POINTER(i32), dp]),
        "cs_autotune_set": (ctypes.c_int, [vp, i32, i32, i32]),
        "cs_wait": (ctypes.c_int, [vp, i64, vp, dp, dp]),
        "cs_req_free": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


EXPORTED = ("cs_ctx_create", "cs_ctx_destroy", "cs_net_create", "cs_net_destroy",
            "cs_opts_default", "cs_screen", "cs_screen_device", "cs_detail",
            "cs_dense_solve_batched", "cs_eigvals_batched", "cs_kkt_at", "cs_stats_get",
            "cs_stats_reset", "cs_last_error", "cs_abi_version", "cs_server_create",
            "cs_server_destroy", "cs_submit", "cs_wait", "cs_req_free", "cs_screen_detail",
            "cs_dyn_at", "cs_screen_device_noalloc", "cs_risk_opts_default", "cs_risk",
            "cs_risk_mc", "cs_screen3_device", "cs_screen_n3_device", "cs_submit_snapshot",
            "cs_server_create_multi", "cs_server_slots", "cs_submit_net", "cs_autotune",
            "cs_autotune_set")


def _check(rc):
    if rc != CS_OK:
        raise CSError(rc, library().cs_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def default_options(**kw) -> Options:
    o = Options()
    library().cs_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Context:
    """A device context (cs_ctx)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self._h = ctypes.c_void_p()
        # networks and servers made on this context: closed before it, also
        # when the garbage collector finalises them in another order
        self._children = weakref.WeakSet()
        _check(library().cs_ctx_create(device, hbm_budget, ctypes.byref(self._h)))

    def close(self):
        if self._h:
            kids = list(self._children)
            for k in [k for k in kids if isinstance(k, Server)] + \
                     [k for k in kids if not isinstance(k, Server)]:
                k.close()
            library().cs_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def stats(self) -> dict:
        st = Stats()
        _check(library().cs_stats_get(self._h, ctypes.byref(st)))
        out = {k: dict(ms=st.ms[i], launches=st.launches[i], units=st.units[i])
               for i, k in enumerate(KERNELS)}
        out["kkt_order"] = st.kkt_order
        out["dyn_order"] = st.dyn_order
        return out

    def reset_stats(self):
        _check(library().cs_stats_reset(self._h))

    def autotune(self, n: int, prec: int = 0, batch: int = 512):
        """Time the batched LU's launch variants for order n (cs_autotune):
        (chosen variant, ms).  Orders up to REG_ORDER: REG_TUNE_VARIANTS in
        ms[0:2] (4 only up to REG_ORDER_W4; NaN where not timed); above:
        TUNE_VARIANTS in ms[0:5]."""
        choice = ctypes.c_int32(0)
        ms = np.zeros(len(TUNE_VARIANTS))
        _check(library().cs_autotune(self.handle, int(n), int(prec), int(batch),
                                     ctypes.byref(choice), _ptr(ms)))
        return int(choice.value), ms

    def autotune_set(self, n: int, prec: int, choice: int):
        """Install a launch variant for order n (REG_TUNE_VARIANTS up to
        REG_ORDER, TUNE_VARIANTS above; 0 = default)."""
        _check(library().cs_autotune_set(self.handle, int(n), int(prec), int(choice)))

    # kernel-level entry points (device pointers, e.g. torch tensors' data_ptr)
    def dense_solve_batched(self, a_ptr, n, nrhs, lda, batch, info_ptr=None, stream=None):
        _check(library().cs_dense_solve_batched(self._h, a_ptr, n, nrhs, lda, batch,
                                                info_ptr, stream))

    def eigvals_batched(self, a_ptr, n, lda, batch, wr_ptr, wi_ptr, info_ptr=None, stream=None):
        _check(library().cs_eigvals_batched(self._h, a_ptr, n, lda, batch, wr_ptr, wi_ptr,
                                            info_ptr, stream))


_F64 = ("vmin", "vmax", "gs", "bs", "br_r", "br_x", "br_b", "br_rate", "br_tap", "br_shift",
        "pmin", "pmax", "qmin", "qmax", "c2", "c1", "c0", "dyn", "pd", "qd")
_I32 = ("br_from", "br_to", "gen_bus", "gen_kind", "load_bus")


class Network:
    """A device-resident network (cs_net) built from a case dict."""

    def __init__(self, ctx: Context, case: dict):
        self.ctx = ctx
        self._keep = {}
        d = _NetDesc()
        for k in ("n_bus", "n_branch", "n_gen", "n_load", "ref_bus"):
            setattr(d, k, int(case[k]))
        d.base_mva = float(case["base_mva"])
        d.f_hz = float(case.get("f_hz", 60.0))
        for k in _F64:
            a = np.ascontiguousarray(case[k], dtype=np.float64)
            self._keep[k] = a
            setattr(d, k, a.ctypes.data)
        for k in _I32:
            a = np.ascontiguousarray(case[k], dtype=np.int32)
            self._keep[k] = a
            setattr(d, k, a.ctypes.data)
        self.n_bus, self.n_branch = int(case["n_bus"]), int(case["n_branch"])
        self.n_gen, self.n_load = int(case["n_gen"]), int(case["n_load"])
        self.n_comp = self.n_branch + self.n_gen + self.n_load
        self._servers = weakref.WeakSet()
        kinds = np.asarray(case.get("gen_kind", np.zeros(self.n_gen)))
        # largest state-matrix order: 7 per machine, 8 per converter, one
        # angle removed
        self.n_states_max = int(np.sum(np.where(kinds == 1, 8, 7))) - 1
        self._h = ctypes.c_void_p()
        _check(library().cs_net_create(ctx.handle, ctypes.byref(d), ctypes.byref(self._h)))
        ctx._children.add(self)

    def close(self):
        if self._h:
            for srv in list(self._servers):
                srv.close()
            library().cs_net_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def screen(self, outages, lam=None, options: Options | None = None):
        """Host buffers in, (records, risk) out."""
        out_list = np.ascontiguousarray(outages, dtype=np.int32).reshape(-1, 2)
        n = len(out_list)
        res = np.zeros(n, dtype=RESULT_DTYPE)
        lam_a = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
        risk = None if lam is None else np.zeros(self.n_comp)
        o = options or default_options()
        _check(library().cs_screen(self.ctx.handle, self._h, _ptr(out_list), n, _ptr(lam_a),
                                   ctypes.byref(o), _ptr(res), _ptr(risk)))
        return res, risk

    def screen_device(self, d_outages, n, d_lambda, d_results, d_risk,
                      options: Options | None = None, stream=None):
        """Device pointers in and out (e.g. torch tensors' data_ptr())."""
        o = options or default_options()
        _check(library().cs_screen_device(self.ctx.handle, self._h, d_outages, n, d_lambda,
                                          ctypes.byref(o), d_results, d_risk, stream))

    def screen_device_noalloc(self, d_outages, n, d_lambda, d_results, d_risk,
                              options: Options | None = None, stream=None):
        """As screen_device, with the workspace in the library's static
        device scratch array: the call allocates no device memory."""
        o = options or default_options()
        _check(library().cs_screen_device_noalloc(self.ctx.handle, self._h, d_outages, n,
                                                  d_lambda, ctypes.byref(o), d_results, d_risk,
                                                  stream))

    def screen3_device(self, d_outages, n, d_lambda, d_results, d_risk,
                       options: Options | None = None, stream=None):
        """Rows of three component ids (N-3; -1 pads N-1/N-2 rows)."""
        o = options or default_options()
        _check(library().cs_screen3_device(self.ctx.handle, self._h, d_outages, n, d_lambda,
                                           ctypes.byref(o), d_results, d_risk, stream))

    def screen_n3_device(self, d_rows, n, d_sub, n_sub, d_sub_records, d_lambda, d_results,
                         d_risk, options: Options | None = None, stream=None) -> int:
        """N-3 rows with pruning by a screened N-1/N-2 list; returns the
        number of rows actually solved."""
        o = options or default_options()
        solved = ctypes.c_int64(0)
        _check(library().cs_screen_n3_device(self.ctx.handle, self._h, d_rows, n, d_sub, n_sub,
                                             d_sub_records, d_lambda, ctypes.byref(o),
                                             d_results, d_risk, ctypes.byref(solved), stream))
        return int(solved.value)

    @staticmethod
    def _risk_opts(severity, zeta_ref, cc_pairs, cc_rate):
        r = RiskOptions()
        library().cs_risk_opts_default(ctypes.byref(r))
        r.severity = severity
        if zeta_ref is not None:
            r.zeta_ref = zeta_ref
        keep = []
        if cc_pairs is not None and len(cc_pairs):
            p = np.ascontiguousarray(cc_pairs, dtype=np.int32).reshape(-1, 2)
            q = np.ascontiguousarray(cc_rate, dtype=np.float64).reshape(-1)
            keep = [p, q]
            r.n_cc, r.cc_pairs, r.cc_rate = len(p), p.ctypes.data, q.ctypes.data
        return r, keep

    def risk(self, d_outages, n, d_records, d_lambda, d_risk, severity=SEV_BINARY,
             zeta_ref=None, cc_pairs=None, cc_rate=None, stream=None):
        """R_i from screened records (device pointers), with the non-binary
        severity and common-cause options."""
        r, keep = self._risk_opts(severity, zeta_ref, cc_pairs, cc_rate)
        _check(library().cs_risk(self.ctx.handle, self._h, d_outages, n, d_records, d_lambda,
                                 ctypes.byref(r), d_risk, stream))
        del keep

    def risk_mc(self, d_outages, n, d_records, d_samples, n_samples, d_risk=None,
                d_moments=None, d_rank_q=None, severity=SEV_BINARY, zeta_ref=None,
                cc_pairs=None, cc_rate=None, stream=None):
        """Monte-Carlo over sampled failure rates (device pointers)."""
        r, keep = self._risk_opts(severity, zeta_ref, cc_pairs, cc_rate)
        _check(library().cs_risk_mc(self.ctx.handle, self._h, d_outages, n, d_records,
                                    d_samples, n_samples, ctypes.byref(r), d_risk, d_moments,
                                    d_rank_q, stream))
        del keep

    def kkt_at(self, outage, iters: int):
        """KKT system and iterate after ``iters`` Newton steps (parity/debug)."""
        nb, nl, ng = self.n_bus, self.n_branch, self.n_gen
        nk = 4 * nb + 2 * ng
        K = np.zeros((nk, nk + 1))
        x = np.zeros(2 * nb + 2 * ng)
        lam = np.zeros(2 * nb)
        z = np.zeros(2 * nl + 2 * nb + 4 * ng)
        mu = np.zeros_like(z)
        met = np.zeros(8)
        status = np.zeros(1, np.int32)
        order = np.zeros(1, np.int32)
        o2 = np.ascontiguousarray(outage, dtype=np.int32).reshape(2)
        _check(library().cs_kkt_at(self.ctx.handle, self._h, _ptr(o2), int(iters), _ptr(K),
                                   _ptr(x), _ptr(lam), _ptr(z), _ptr(mu), _ptr(met),
                                   _ptr(status), _ptr(order)))
        return dict(K=K[:, :nk].copy(), rhs=K[:, nk].copy(), x=x, lam=lam, z=z, mu=mu,
                    metrics=met, status=int(status[0]))

    def detail(self, outage, options: Options | None = None):
        o = options or default_options()
        rec = np.zeros(1, dtype=RESULT_DTYPE)
        vm = np.zeros(self.n_bus)
        va = np.zeros(self.n_bus)
        pg = np.zeros(self.n_gen)
        qg = np.zeros(self.n_gen)
        er = np.zeros(self.n_states_max)
        ei = np.zeros(self.n_states_max)
        ne = np.zeros(1, dtype=np.int32)
        lab = np.zeros(self.n_bus, dtype=np.int32)
        o2 = np.ascontiguousarray(outage, dtype=np.int32).reshape(2)
        _check(library().cs_detail(self.ctx.handle, self._h, _ptr(o2), ctypes.byref(o),
                                   _ptr(rec), _ptr(vm), _ptr(va), _ptr(pg), _ptr(qg),
                                   _ptr(er), _ptr(ei), _ptr(ne), _ptr(lab)))
        k = int(ne[0])
        return dict(record=rec[0], vm=vm, va=va, pg=pg, qg=qg,
                    eig=er[:k] + 1j * ei[:k], label=lab)


    def screen_detail(self, outages, options: Options | None = None):
        """Records plus each scenario's operating point and spectrum
        (parity checks): dict of records, vm, va [n][n_bus], pg, qg
        [n][n_gen], eig (list of complex arrays)."""
        out_list = np.ascontiguousarray(outages, dtype=np.int32).reshape(-1, 2)
        n = len(out_list)
        nb, ng = self.n_bus, self.n_gen
        na = self.n_states_max
        res = np.zeros(n, dtype=RESULT_DTYPE)
        vm, va = np.zeros((n, nb)), np.zeros((n, nb))
        pg, qg = np.zeros((n, ng)), np.zeros((n, ng))
        er, ei = np.zeros((n, na)), np.zeros((n, na))
        ne = np.zeros(n, dtype=np.int32)
        o = options or default_options()
        _check(library().cs_screen_detail(self.ctx.handle, self._h, _ptr(out_list), n,
                                          ctypes.byref(o), _ptr(res), _ptr(vm), _ptr(va),
                                          _ptr(pg), _ptr(qg), _ptr(er), _ptr(ei), _ptr(ne)))
        eig = [er[i, :ne[i]] + 1j * ei[i, :ne[i]] for i in range(n)]
        return dict(records=res, vm=vm, va=va, pg=pg, qg=qg, eig=eig, n_eig=ne)

    def dyn_at(self, outage, vm, va, pg, qg, eigenvalues: bool = True):
        """State matrix (row-major) and its eigenvalues at a given operating
        point over the whole network (only the island's entries are read)."""
        na = self.n_states_max
        A = np.zeros(na * na)
        er, ei = np.zeros(na), np.zeros(na)
        ns = np.zeros(1, dtype=np.int32)
        o2 = np.ascontiguousarray(outage, dtype=np.int32).reshape(2)
        arr = [np.ascontiguousarray(v, dtype=np.float64) for v in (vm, va, pg, qg)]
        _check(library().cs_dyn_at(self.ctx.handle, self._h, _ptr(o2), *[_ptr(v) for v in arr],
                                   _ptr(A), _ptr(ns), _ptr(er) if eigenvalues else None,
                                   _ptr(ei) if eigenvalues else None))
        k = int(ns[0])
        return A[:k * k].reshape(k, k).copy(), (er[:k] + 1j * ei[:k]) if eigenvalues else None


class Request:
    """One submitted screening request (cs_req)."""

    def __init__(self, server: "Server", handle, n: int, has_lam: bool, n_comp: int):
        self.server = server
        self._h = handle
        self.n = n
        self.has_lam = has_lam
        self.n_comp = n_comp

    def wait(self, timeout_s: float | None = None):
        """(records, risk or None, latency_s); raises CSError(CS_ETIMEDOUT)."""
        res = np.zeros(self.n, dtype=RESULT_DTYPE)
        risk = np.zeros(self.n_comp) if self.has_lam else None
        lat = np.zeros(1)
        us = -1 if timeout_s is None else int(timeout_s * 1e6)
        _check(library().cs_wait(self._h, us, _ptr(res), _ptr(risk), _ptr(lat)))
        return res, risk, float(lat[0])

    def close(self):
        if self._h:
            library().cs_req_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A serving engine (cs_server) for one network, or for several under
    one HBM budget (``net`` a list; ``shares`` their parts of the budget):
    requests are admitted as slots free up and run beside each other on the
    device."""

    def __init__(self, ctx: Context, net, options: Options | None = None,
                 queue_capacity: int = 1 << 18, shares=None):
        self.ctx = ctx
        self.nets = list(net) if isinstance(net, (list, tuple)) else [net]
        self.net = self.nets[0]
        self._h = ctypes.c_void_p()
        o = options or default_options()
        handles = (ctypes.c_void_p * len(self.nets))(*[n._h for n in self.nets])
        sh = None if shares is None else np.ascontiguousarray(shares, dtype=np.float64)
        if sh is not None and len(sh) != len(self.nets):
            raise ValueError("one share per network")
        _check(library().cs_server_create_multi(ctx.handle, handles, len(self.nets), _ptr(sh),
                                                ctypes.byref(o), int(queue_capacity),
                                                ctypes.byref(self._h)))
        ctx._children.add(self)
        for n in self.nets:
            n._servers.add(self)

    def slots(self, net: int = 0) -> int:
        rc = library().cs_server_slots(self._h, int(net))
        _check(rc if rc < 0 else CS_OK)
        return rc

    def submit(self, outages, lam=None, load_scale=None, net: int = 0) -> Request:
        """Admit a request for network ``net``; load_scale [n_load] screens it
        on a snapshot of the network with every load scaled by its factor."""
        out_list = np.ascontiguousarray(outages, dtype=np.int32).reshape(-1, 2)
        lam_a = None if lam is None else np.ascontiguousarray(lam, dtype=np.float64)
        sc = None if load_scale is None else np.ascontiguousarray(load_scale, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(library().cs_submit_net(self._h, int(net), _ptr(out_list), len(out_list),
                                       _ptr(lam_a), _ptr(sc), ctypes.byref(h)))
        n_comp = self.nets[net].n_comp if 0 <= net < len(self.nets) else 0
        return Request(self, h, len(out_list), lam is not None, n_comp)

    def close(self):
        if self._h:
            library().cs_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

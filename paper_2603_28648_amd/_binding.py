"""ctypes binding of the C ABI in include/dmrg.h (argument marshalling only).

Every computation runs in the HIP library ``libdmrg_mi355x.so``; this module
only converts Python / NumPy / torch arguments to pointers and status codes
to exceptions.  There is no fallback: if the library is missing or no GPU is
present, the calls raise.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmrg_mi355x.so")

DMRG_FP64, DMRG_BF16, DMRG_BF16X3, DMRG_OZAKI = 0, 1, 2, 3
PRECISIONS = {"fp64": DMRG_FP64, "bf16": DMRG_BF16, "bf16x3": DMRG_BF16X3, "ozaki": DMRG_OZAKI}

STATUS = {0: "OK", 1: "WARN_NOT_CONVERGED", -1: "INVALID_ARG", -2: "SHAPE", -3: "HIP",
          -4: "OOM", -5: "NO_DEVICE", -6: "UNIMPLEMENTED", -7: "STATE"}


class DMRGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)} ({status}): {msg}")
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [("n_orb", ctypes.c_int32), ("n_elec", ctypes.c_int32),
                ("two_sz", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("e_core", ctypes.c_double),
                ("h", ctypes.POINTER(ctypes.c_double)),
                ("eri", ctypes.POINTER(ctypes.c_double))]


class Mps(ctypes.Structure):
    _fields_ = [("n_sites", ctypes.c_int32), ("window", ctypes.c_int32),
                ("bond_offsets", ctypes.POINTER(ctypes.c_int32)),
                ("sector_n", ctypes.POINTER(ctypes.c_int32)),
                ("sector_2sz", ctypes.POINTER(ctypes.c_int32)),
                ("sector_dim", ctypes.POINTER(ctypes.c_int32)),
                ("site_data", ctypes.POINTER(ctypes.POINTER(ctypes.c_double)))]


class SigmaInfo(ctypes.Structure):
    _fields_ = [("flops", ctypes.c_double), ("hw_flops", ctypes.c_double),
                ("n_pairs", ctypes.c_int64), ("n_right_ops", ctypes.c_int64),
                ("n_stage1_tiles", ctypes.c_int64), ("n_stage2_tiles", ctypes.c_int64),
                ("n_stage2_segments", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("operator_bytes", ctypes.c_int64), ("n_chunks", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("flops_stage1", ctypes.c_double),
                ("flops_stage2", ctypes.c_double), ("bf_config_stage1", ctypes.c_int32),
                ("bf_config_stage2", ctypes.c_int32), ("tune_ms", ctypes.c_double),
                ("flops_terms", ctypes.c_double), ("flops_stage1_used", ctypes.c_double)]


class DavidsonOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("max_subspace", ctypes.c_int32),
                ("tol", ctypes.c_double), ("n_ladder", ctypes.c_int32),
                ("ladder", ctypes.c_int32 * 4), ("ladder_tol", ctypes.c_double * 4),
                ("precondition", ctypes.c_int32), ("restart", ctypes.c_int32),
                ("refine", ctypes.c_int32)]


class SigmaTimes(ctypes.Structure):
    _fields_ = [("calls", ctypes.c_int32), ("launches_stage1", ctypes.c_int32),
                ("launches_stage2", ctypes.c_int32), ("launches_pinned", ctypes.c_int32),
                ("ms_stage1", ctypes.c_double), ("ms_stage2", ctypes.c_double),
                ("ms_pinned", ctypes.c_double), ("flops_stage1", ctypes.c_double),
                ("flops_stage2", ctypes.c_double), ("flops_pinned", ctypes.c_double),
                ("launches_convert", ctypes.c_int32), ("pad", ctypes.c_int32), ("ms_convert", ctypes.c_double)]


class DavidsonStats(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_double), ("residual", ctypes.c_double),
                ("time_ms", ctypes.c_double), ("sigma_ms", ctypes.c_double),
                ("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("n_sigma", ctypes.c_int32 * 4), ("n_history", ctypes.c_int32),
                ("residual_history", ctypes.c_double * 256),
                ("stage_history", ctypes.c_int32 * 256)]


class Su2Window(ctypes.Structure):
    _fields_ = [("n_left", ctypes.c_int32), ("n_right", ctypes.c_int32),
                ("left_n", ctypes.POINTER(ctypes.c_int32)), ("left_two_s", ctypes.POINTER(ctypes.c_int32)),
                ("left_dim", ctypes.POINTER(ctypes.c_int32)), ("right_n", ctypes.POINTER(ctypes.c_int32)),
                ("right_two_s", ctypes.POINTER(ctypes.c_int32)), ("right_dim", ctypes.POINTER(ctypes.c_int32)),
                ("n_elec", ctypes.c_int32), ("two_s", ctypes.c_int32)]


class Su2Operator(ctypes.Structure):
    _fields_ = [("n_blocks", ctypes.c_int32), ("out_sector", ctypes.POINTER(ctypes.c_int32)),
                ("in_sector", ctypes.POINTER(ctypes.c_int32)), ("offset", ctypes.POINTER(ctypes.c_int64)),
                ("data", ctypes.c_void_p)]


class Su2Info(ctypes.Structure):
    _fields_ = [("psi_size", ctypes.c_int64), ("n_chunks", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("n_segments", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64),
                ("flops_stage1", ctypes.c_double), ("flops_stage2", ctypes.c_double)]


class Su2Basis(ctypes.Structure):
    _fields_ = [("n_coupled", ctypes.c_int32), ("coupled_dim", ctypes.POINTER(ctypes.c_int32)),
                ("coupled_group", ctypes.POINTER(ctypes.c_int32)), ("n_groups", ctypes.c_int32),
                ("group_dim", ctypes.POINTER(ctypes.c_int32)), ("proj", ctypes.POINTER(ctypes.c_void_p))]


class Su2Pair(ctypes.Structure):
    _fields_ = [("left_op", ctypes.c_int32), ("right_op", ctypes.c_int32), ("two_k", ctypes.c_int32),
                ("parity", ctypes.c_int32), ("coef", ctypes.c_double)]


EXPORTS = {
    "dmrg_create": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_void_p]),
    "dmrg_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "dmrg_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "dmrg_build_ops": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.POINTER(Mps),
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32]),
    "dmrg_psi_size": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "dmrg_sigma": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "dmrg_sigma_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "dmrg_sigma_get_info": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(SigmaInfo)]),
    "dmrg_davidson": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(DavidsonOpts),
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(DavidsonStats)]),
    "dmrg_truncate": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "dmrg_get_psi": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "dmrg_sigma_timing": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(SigmaTimes)]),
    "dmrg_sigma_graphs": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "dmrg_orbital_gradient": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p]),
    "dmrg_sigma_backward": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "dmrg_debug_diag": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "dmrg_validate": (ctypes.c_int32, [ctypes.POINTER(Problem), ctypes.POINTER(Mps)]),
    "dmrg_get_bond": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "dmrg_get_site": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "dmrg_energy": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_int32,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]),
    "dmrg_su2_psi_size": (ctypes.c_int32, [ctypes.POINTER(Su2Window), ctypes.POINTER(ctypes.c_int64)]),
    "dmrg_su2_sigma": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Su2Window), ctypes.c_int32,
                                        ctypes.POINTER(Su2Operator), ctypes.c_int32, ctypes.POINTER(Su2Operator),
                                        ctypes.c_int32, ctypes.POINTER(Su2Pair), ctypes.c_void_p, ctypes.c_void_p]),
    "dmrg_su2_plan_create": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Su2Window), ctypes.c_int32,
                                              ctypes.POINTER(Su2Operator), ctypes.c_int32,
                                              ctypes.POINTER(Su2Operator), ctypes.c_int32, ctypes.POINTER(Su2Pair),
                                              ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "dmrg_su2_plan_sigma": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "dmrg_su2_plan_info": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Su2Info)]),
    "dmrg_su2_plan_destroy": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "dmrg_su2_product_size": (ctypes.c_int32, [ctypes.POINTER(Su2Window), ctypes.POINTER(Su2Operator),
                                               ctypes.POINTER(Su2Operator), ctypes.c_int32, ctypes.c_int32,
                                               ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                               ctypes.POINTER(ctypes.c_int64)]),
    "dmrg_su2_product": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Su2Window), ctypes.POINTER(Su2Operator),
                                          ctypes.POINTER(Su2Operator), ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.c_void_p]),
    "dmrg_su2_rotate_size": (ctypes.c_int32, [ctypes.POINTER(Su2Basis), ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int64)]),
    "dmrg_su2_rotate": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(Su2Basis), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "dmrg_debug_gemm": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_int32, ctypes.c_double,
                                         ctypes.c_int32, ctypes.c_int32]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(
            f"{path} is missing: build it with `python -m paper_2603_28648_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _dev_ptr(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _problem(h, eri, n_elec, two_sz, e_core, keep):
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    keep += [h, eri]
    return Problem(h.shape[0], int(n_elec), int(two_sz), 0, float(e_core), _ptr(h), _ptr(eri))


def _mps(mps_arrays, window, keep):
    a = mps_arrays
    K = len(a["sites"])
    arrs = [np.ascontiguousarray(a[k], dtype=np.int32)
            for k in ("bond_offsets", "sector_n", "sector_2sz", "sector_dim")]
    keep += arrs
    ptrs = (ctypes.POINTER(ctypes.c_double) * K)()
    for b, s in enumerate(a["sites"]):
        if s is not None:
            s = np.ascontiguousarray(s, dtype=np.float64)
            keep.append(s)
            ptrs[b] = _ptr(s)
    keep.append(ptrs)
    return Mps(K, int(window), *[_ptr(x, ctypes.c_int32) for x in arrs],
               ctypes.cast(ptrs, ctypes.POINTER(ctypes.POINTER(ctypes.c_double))))


def _su2_window(left_sectors, right_sectors, n_elec, two_s, keep):
    """left_sectors / right_sectors: lists of (N, 2S, dimension)."""
    cols = []
    for secs in (left_sectors, right_sectors):
        a = np.asarray(secs, dtype=np.int32).reshape(-1, 3)
        cols += [np.ascontiguousarray(a[:, i]) for i in range(3)]
    keep += cols
    return Su2Window(len(left_sectors), len(right_sectors), *[_ptr(c, ctypes.c_int32) for c in cols],
                     int(n_elec), int(two_s))


def su2_psi_size(left_sectors, right_sectors, n_elec, two_s):
    """Length of the reduced spin-adapted window vector (dmrg_su2_psi_size; no GPU)."""
    lib = load_library()
    keep = []
    w = _su2_window(left_sectors, right_sectors, n_elec, two_s, keep)
    n = ctypes.c_int64()
    st = lib.dmrg_su2_psi_size(ctypes.byref(w), ctypes.byref(n))
    if st < 0:
        raise DMRGError(st, lib.dmrg_last_error(None).decode())
    return n.value


class Su2Plan:
    """A spin-adapted sigma planned once (dmrg_su2_plan_*).  sigma(psi, out)
    is stream-ordered on the context stream; close() (or leaving a with
    block) synchronises and releases the plan."""

    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h

    def sigma(self, psi, out):
        n = self.info()["psi_size"]
        if psi.numel() != n or out.numel() != n:
            raise ValueError(f"expected {n} elements, got {psi.numel()} and {out.numel()}")
        self.ctx._check(self.ctx.lib.dmrg_su2_plan_sigma(self.ctx.h, self.h, _dev_ptr(psi), _dev_ptr(out)),
                        self.ctx.h)
        return out

    def info(self):
        o = Su2Info()
        self.ctx._check(self.ctx.lib.dmrg_su2_plan_info(self.ctx.h, self.h, ctypes.byref(o)), self.ctx.h)
        return {"psi_size": o.psi_size, "n_chunks": o.n_chunks, "n_segments": o.n_segments,
                "workspace_bytes": o.workspace_bytes, "flops_stage1": o.flops_stage1,
                "flops_stage2": o.flops_stage2}

    def close(self):
        if self.h and getattr(self.ctx, "h", None):
            self.ctx._check(self.ctx.lib.dmrg_su2_plan_destroy(self.ctx.h, self.h), self.ctx.h)
        self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def validate(h, eri, n_elec, two_sz, mps_arrays=None, window=0, e_core=0.0):
    """Host-side check of a problem (and MPS layout) by dmrg_validate; needs no
    GPU.  Raises DMRGError with the library's status and message."""
    lib = load_library()
    keep = []
    prob = _problem(h, eri, n_elec, two_sz, e_core, keep)
    mps = _mps(mps_arrays, window, keep) if mps_arrays is not None else None
    st = lib.dmrg_validate(ctypes.byref(prob), ctypes.byref(mps) if mps is not None else None)
    if st < 0:
        raise DMRGError(st, lib.dmrg_last_error(None).decode())
    return st


class Context:
    """One library context on one GPU, ordered on torch's current stream."""

    def __init__(self, device=0, stream=None):
        self.lib = load_library()
        if stream is None:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        h = ctypes.c_void_p()
        self._check(self.lib.dmrg_create(ctypes.byref(h), int(device), ctypes.c_void_p(stream)), None)
        self.h = h
        self._keep = []

    def _check(self, st, h):
        if st < 0:
            raise DMRGError(st, self.lib.dmrg_last_error(h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            self.lib.dmrg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_ops(self, site, direction=0, h=None, eri=None, n_elec=None, two_sz=None,
                  mps_arrays=None, window=None, e_core=0.0, precision_mask=1):
        prob = None
        keep = []
        if h is not None:
            self._n_orb = int(np.asarray(h).shape[0])
            self._e_core = float(e_core)
            prob = _problem(h, eri, n_elec, two_sz, e_core, keep)
        mps = None
        if mps_arrays is not None:
            mps = _mps(mps_arrays, site if window is None else window, keep)
        st = self.lib.dmrg_build_ops(self.h, ctypes.byref(prob) if prob else None,
                                     ctypes.byref(mps) if mps else None, int(site), int(direction),
                                     int(precision_mask))
        self._check(st, self.h)
        self._window = int(site)
        return st

    def psi_size(self):
        n = ctypes.c_int64()
        self._check(self.lib.dmrg_psi_size(self.h, ctypes.byref(n)), self.h)
        return n.value

    def sigma(self, psi, out, precision="fp64"):
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self._check(self.lib.dmrg_sigma(self.h, _dev_ptr(psi), _dev_ptr(out), p), self.h)
        return out

    def sigma_noalloc(self, psi, out):
        """FP64 sigma through dmrg_sigma_noalloc (no device allocation)."""
        self._check(self.lib.dmrg_sigma_noalloc(self.h, _dev_ptr(psi), _dev_ptr(out)), self.h)
        return out

    def orbital_gradient(self, dh, deri):
        """Generalised Fock matrix and orbital gradient dE/dkappa (K x K each)
        from the backward's dh, deri and the loaded integrals."""
        import torch
        fock = torch.empty_like(dh)
        grad = torch.empty_like(dh)
        self._check(self.lib.dmrg_orbital_gradient(self.h, _dev_ptr(dh.contiguous()), _dev_ptr(deri.contiguous()),
                                                   _dev_ptr(fock), _dev_ptr(grad)), self.h)
        return fock, grad

    def sigma_graphs(self, enable=True):
        """Replay every sigma of this context from a captured HIP graph."""
        self._check(self.lib.dmrg_sigma_graphs(self.h, int(bool(enable))), self.h)

    def sigma_timing(self, mode=-1):
        """Kernel timing of sigma calls (mode 1: reset and start, 0: stop,
        -1: keep); returns the totals so far as a dict."""
        t = SigmaTimes()
        self._check(self.lib.dmrg_sigma_timing(self.h, int(mode), ctypes.byref(t)), self.h)
        return {k: getattr(t, k) for k, _ in SigmaTimes._fields_}

    def sigma_backward(self, psi, sigma_bar=None, dh=None, deri=None, precision="fp64"):
        """Gradient of <sigma_bar, H_eff psi> with respect to h (K x K) and
        (pq|rs) (K^4): the transition 1-RDM and half the 2-RDM.  precision
        "bf16x3" (or "bf16") runs the adjoint contractions on the BF16 kernel."""
        import torch
        K = self._n_orb
        if dh is None:
            dh = torch.empty((K, K), dtype=torch.float64, device=psi.device)
        if deri is None:
            deri = torch.empty((K, K, K, K), dtype=torch.float64, device=psi.device)
        lam = ctypes.c_void_p(None) if sigma_bar is None else _dev_ptr(sigma_bar)
        self._check(self.lib.dmrg_sigma_backward(self.h, _dev_ptr(psi), lam, _dev_ptr(dh), _dev_ptr(deri),
                                                 PRECISIONS[precision] if isinstance(precision, str) else int(precision)),
                    self.h)
        return dh, deri

    def davidson(self, psi, tol=1e-6, max_iter=100, max_subspace=24,
                 ladder=(("fp64", None),), precondition=2, restart=6, refine=False):
        """Lowest eigenpair at the current window; psi (device) is updated in place.

        ladder: sequence of (precision, stage-end residual); the last stage
        must be fp64 (its threshold is tol).  refine: in the last stage, each
        correction vector solves the Jacobi-Davidson correction equation for
        the FP64 residual with the previous stage's reduced precision."""
        o = DavidsonOpts()
        o.max_iter, o.max_subspace, o.tol = int(max_iter), int(max_subspace), float(tol)
        o.n_ladder = len(ladder)
        o.precondition = int(precondition)
        o.restart = int(restart)
        o.refine = int(bool(refine))
        for k, (p, t) in enumerate(ladder):
            o.ladder[k] = PRECISIONS[p] if isinstance(p, str) else int(p)
            o.ladder_tol[k] = float(t) if t is not None else 0.0
        e = ctypes.c_double()
        st = DavidsonStats()
        status = self.lib.dmrg_davidson(self.h, _dev_ptr(psi), ctypes.byref(o), ctypes.byref(e),
                                        ctypes.byref(st))
        self._check(status, self.h)
        n = st.n_history
        return {"energy": e.value, "residual": st.residual, "time_ms": st.time_ms,
                "sigma_ms": st.sigma_ms, "iterations": st.iterations,
                "converged": bool(st.converged), "status": status,
                "n_sigma": {"fp64": st.n_sigma[0], "bf16": st.n_sigma[1], "bf16x3": st.n_sigma[2],
                            "ozaki": st.n_sigma[3]},
                "residual_history": list(st.residual_history[:n]),
                "stage_history": list(st.stage_history[:n])}

    def truncate(self, psi, direction, max_bond_dim, cutoff=0.0):
        """Truncate the window and move it; returns (truncation error, kept bond dimension)."""
        e = ctypes.c_double()
        k = ctypes.c_int32()
        self._check(self.lib.dmrg_truncate(self.h, _dev_ptr(psi), int(direction), int(max_bond_dim),
                                           float(cutoff), ctypes.byref(e), ctypes.byref(k)), self.h)
        return e.value, k.value

    def get_psi(self, out):
        self._check(self.lib.dmrg_get_psi(self.h, _dev_ptr(out)), self.h)
        return out

    def _half_sweeps(self, psi, n_half, max_bond_dim, tol, ladder, log, refine=False, max_iter=100):
        """n_half half-sweeps from the loaded window; per half-sweep: energy of
        its last window, lowest energy, largest truncation error, the seconds
        spent in the eigensolver and in operator construction, and one record
        per window of its eigensolver result (converged, iterations,
        residual): a window that stops at max_iter without reaching tol is
        counted in "unconverged", never silently dropped."""
        import time
        import torch
        K = self._n_orb
        out = []
        cur = psi
        site = self._window
        direction = -1 if site == K - 2 else +1
        for _ in range(n_half):
            e_last, e_min, eps_max, t_dav, t_build = None, np.inf, 0.0, 0.0, 0.0
            windows = []
            while True:
                t0 = time.perf_counter()
                r = self.davidson(cur, tol=tol, ladder=ladder, refine=refine, max_iter=max_iter)
                torch.cuda.synchronize()
                t_dav += time.perf_counter() - t0
                e_last = r["energy"]
                e_min = min(e_min, e_last)
                windows.append({"window": site, "converged": r["converged"], "iterations": r["iterations"],
                                "residual": r["residual"]})
                at_end = (direction > 0 and site == K - 2) or (direction < 0 and site == 0)
                move = -direction if at_end else direction
                eps, kept = self.truncate(cur, move, max_bond_dim)
                eps_max = max(eps_max, eps)
                site += move
                t0 = time.perf_counter()
                self.build_ops(site, move)
                torch.cuda.synchronize()
                t_build += time.perf_counter() - t0
                cur = torch.empty(self.psi_size(), dtype=torch.float64, device=cur.device)
                self.get_psi(cur)
                if log:
                    log(f"window {site - move} E={e_last:.12f} eps={eps:.2e} D={kept} "
                        f"residual={r['residual']:.1e}{'' if r['converged'] else ' (not converged)'}")
                if at_end:
                    direction = move
                    break
            out.append({"energy": e_last, "min_energy": e_min, "max_trunc": eps_max,
                        "davidson_s": t_dav, "build_s": t_build, "windows": windows,
                        "unconverged": sum(1 for w in windows if not w["converged"])})
        return out, cur

    def sweep(self, psi, n_sweeps, max_bond_dim, tol=1e-6, ladder=(("fp64", None),), log=None,
              refine=False, max_iter=100):
        """Two-site sweeps from the loaded window; returns per-half-sweep
        energies, largest truncation errors, and the final window vector.

        psi: device tensor of the current window; the context's window must be
        0 (start of a left-to-right sweep).  Each half-sweep optimises every
        window once and turns at the chain end."""
        halves, cur = self._half_sweeps(psi, 2 * n_sweeps, max_bond_dim, tol, ladder, log, refine, max_iter)
        self.last_halves = halves
        return [h["energy"] for h in halves], [h["max_trunc"] for h in halves], cur

    def sweep_to_convergence(self, psi, max_bond_dim, sweep_tol=1e-5, max_sweeps=20, tol=1e-6,
                             ladder=(("fp64", None),), log=None, refine=False, max_iter=100,
                             require_converged=False):
        """Full sweeps (there and back) until the energies of three subsequent
        sweeps agree within sweep_tol (the paper's stopping rule, 1e-5 Ha).
        E_s is the lowest energy met in sweep s, eps_s its largest truncation
        error.  Returns a dict with the per-sweep records (each with the count
        of windows whose eigensolver stopped at max_iter before tol), whether
        the rule was met, the total of such windows, and the final window
        vector.  log (optional) receives one line per sweep.  refine: residual
        refinement in every window's eigensolver (see davidson).
        require_converged: raise RuntimeError when a window's eigensolver
        does not converge."""
        from .extrapolate import sweep_converged
        sweeps = []
        cur = psi
        while len(sweeps) < max_sweeps:
            halves, cur = self._half_sweeps(cur, 2, max_bond_dim, tol, ladder, None, refine, max_iter)
            sweeps.append({"min_energy": min(h["min_energy"] for h in halves),
                           "max_trunc": max(h["max_trunc"] for h in halves),
                           "davidson_s": sum(h["davidson_s"] for h in halves),
                           "build_s": sum(h["build_s"] for h in halves),
                           "unconverged": sum(h["unconverged"] for h in halves),
                           "max_residual": max(w["residual"] for h in halves for w in h["windows"])})
            sw = sweeps[-1]
            if log:
                log(f"sweep {len(sweeps)}: E={sw['min_energy']:.12f} eps={sw['max_trunc']:.2e} "
                    f"eigensolver {sw['davidson_s']:.1f} s, operators {sw['build_s']:.1f} s, "
                    f"unconverged windows {sw['unconverged']} (largest residual {sw['max_residual']:.1e})")
            if require_converged and sw["unconverged"]:
                raise RuntimeError(f"sweep {len(sweeps)}: {sw['unconverged']} windows did not reach "
                                   f"residual {tol} in {max_iter} iterations")
            if sweep_converged([s_["min_energy"] for s_ in sweeps], sweep_tol):
                break
        converged = sweep_converged([sw["min_energy"] for sw in sweeps], sweep_tol)
        return {"sweeps": sweeps, "converged": converged, "energy": sweeps[-1]["min_energy"],
                "max_trunc": sweeps[-1]["max_trunc"], "psi": cur,
                "unconverged_windows": sum(sw["unconverged"] for sw in sweeps)}

    def get_bond(self, bond):
        """Sectors of a bond of the context's MPS: list of (N, 2Sz, dim)."""
        n = ctypes.c_int32()
        self._check(self.lib.dmrg_get_bond(self.h, int(bond), 0, ctypes.byref(n), None, None, None), self.h)
        a = [np.zeros(max(1, n.value), dtype=np.int32) for _ in range(3)]
        self._check(self.lib.dmrg_get_bond(self.h, int(bond), n.value, ctypes.byref(n),
                                           *[_ptr(x, ctypes.c_int32) for x in a]), self.h)
        return [(int(a[0][k]), int(a[1][k]), int(a[2][k])) for k in range(n.value)]

    def get_site(self, site):
        """The packed site tensor of a site outside the window (host float64
        array in the dmrg_mps layout)."""
        n = ctypes.c_int64()
        self._check(self.lib.dmrg_get_site(self.h, int(site), 0, None, ctypes.byref(n)), self.h)
        out = np.zeros(max(1, n.value), dtype=np.float64)
        self._check(self.lib.dmrg_get_site(self.h, int(site), n.value, _ptr(out), ctypes.byref(n)), self.h)
        return out[:n.value]

    def energy(self, psi, precision="fp64", h=None, eri=None, sigma=None, grad=None):
        """(psi^T H_eff psi + e_core psi^T psi, psi^T psi) from dmrg_energy;
        sigma / grad (device tensors, optional) receive H_eff psi and
        2 (sigma + e_core psi).  h / eri (optional) are checked against the
        integrals the operators were built from."""
        keep = []
        hp = ep = None
        if h is not None:
            hh = np.ascontiguousarray(np.asarray(h, dtype=np.float64))
            ee = np.ascontiguousarray(np.asarray(eri, dtype=np.float64))
            keep += [hh, ee]
            hp, ep = _ptr(hh), _ptr(ee)
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        e = ctypes.c_double()
        nrm = ctypes.c_double()
        self._check(self.lib.dmrg_energy(self.h, hp, ep, _dev_ptr(psi), p,
                                         _dev_ptr(sigma) if sigma is not None else None,
                                         _dev_ptr(grad) if grad is not None else None,
                                         ctypes.byref(e), ctypes.byref(nrm)), self.h)
        return e.value, nrm.value

    def _su2_args(self, left_sectors, right_sectors, n_elec, two_s, left_ops, right_ops, pairs, keep):
        """ctypes arguments of the spin-adapted calls.  Sectors: lists of
        (N, 2S, dimension).  An operator is (blocks, data) or (blocks, data,
        base): blocks a list of (out sector, in sector, element offset), data
        a contiguous float64 CUDA tensor holding the row-major blocks from
        element base on (default 0).  pairs: (left op, right op, 2k, parity of
        the right op, coef)."""
        w = _su2_window(left_sectors, right_sectors, n_elec, two_s, keep)

        def ops(lst, sectors):
            dims = np.asarray([d for _, _, d in sectors], dtype=np.int64)
            arr = (Su2Operator * max(1, len(lst)))()
            for i, op in enumerate(lst):
                blocks, data = op[0], op[1]
                base = int(op[2]) if len(op) > 2 else 0
                b = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
                o, n_, off = (np.ascontiguousarray(b[:, 0], dtype=np.int32),
                              np.ascontiguousarray(b[:, 1], dtype=np.int32), np.ascontiguousarray(b[:, 2]))
                ptr = _dev_ptr(data).value
                if len(b):
                    # every block inside the tensor (the library only sees pointers)
                    if o.min() < 0 or n_.min() < 0 or o.max() >= len(dims) or n_.max() >= len(dims):
                        raise ValueError(f"operator {i}: block sector out of range")
                    end = base + int((off + dims[o] * dims[n_]).max())
                    if base < 0 or off.min() < 0 or end > data.numel():
                        raise ValueError(f"operator {i}: blocks reach past its data tensor")
                keep.extend([o, n_, off, data])
                arr[i] = Su2Operator(len(b), _ptr(o, ctypes.c_int32), _ptr(n_, ctypes.c_int32),
                                     _ptr(off, ctypes.c_int64), ptr + 8 * base)
            return arr

        la, ra = ops(left_ops, left_sectors), ops(right_ops, right_sectors)
        pa = (Su2Pair * max(1, len(pairs)))(*[Su2Pair(int(l), int(r), int(k), int(p), float(c))
                                               for l, r, k, p, c in pairs])
        keep.extend([la, ra, pa])
        return ctypes.byref(w), len(left_ops), la, len(right_ops), ra, len(pairs), pa

    def su2_sigma(self, left_sectors, right_sectors, n_elec, two_s, left_ops, right_ops, pairs, psi, out):
        """dmrg_su2_sigma (arguments as in _su2_args); synchronises."""
        keep = []
        args = self._su2_args(left_sectors, right_sectors, n_elec, two_s, left_ops, right_ops, pairs, keep)
        self._su2_check_vectors(left_sectors, right_sectors, n_elec, two_s, psi, out)
        self._check(self.lib.dmrg_su2_sigma(self.h, *args, _dev_ptr(psi), _dev_ptr(out)), self.h)
        return out

    @staticmethod
    def _su2_check_vectors(left_sectors, right_sectors, n_elec, two_s, *vecs):
        n = su2_psi_size(left_sectors, right_sectors, n_elec, two_s)
        for v in vecs:
            if v.numel() != n:
                raise ValueError(f"expected {n} elements, got {v.numel()}")

    def su2_product(self, sectors1, sectors2, a_op, b_op, tk1, tk2, tk, parity_b):
        """dmrg_su2_product: the reduced blocks of [A^k1 x B^k2]^k (operators
        as in _su2_args, A on the subsystem of sectors1, B on sectors2).
        Returns (blocks [(out coupled sector, in coupled sector, offset)],
        float64 CUDA tensor of the data)."""
        import torch
        keep = []
        wptr, _, la, _, ra, _, _ = self._su2_args(sectors1, sectors2, 0, 0, [a_op], [b_op], [], keep)
        nb, ne = ctypes.c_int32(), ctypes.c_int64()
        self._check(self.lib.dmrg_su2_product_size(wptr, la, ra, int(tk1), int(tk2), int(tk), ctypes.byref(nb),
                                                   ctypes.byref(ne)), None)
        out = np.zeros(max(1, nb.value), dtype=np.int32)
        inn = np.zeros(max(1, nb.value), dtype=np.int32)
        off = np.zeros(max(1, nb.value), dtype=np.int64)
        data = torch.zeros(max(1, ne.value), dtype=torch.float64, device="cuda")
        self._check(self.lib.dmrg_su2_product(self.h, wptr, la, ra, int(tk1), int(tk2), int(tk), int(parity_b),
                                              _ptr(out, ctypes.c_int32), _ptr(inn, ctypes.c_int32),
                                              _ptr(off, ctypes.c_int64), _dev_ptr(data)), self.h)
        return [(int(out[i]), int(inn[i]), int(off[i])) for i in range(nb.value)], data

    def su2_rotate(self, blocks, data, coupled_dims, coupled_group, group_dims, proj):
        """dmrg_su2_rotate: blocks [(out coupled sector, in coupled sector,
        offset)] and their float64 CUDA data (as su2_product returns them),
        the coupled sectors' dimensions and new sectors (-1: kept out), the
        kept dimension of each new sector, and proj[c] a float64 CUDA tensor
        of d_c x D_g (None where kept out).  Returns (blocks [(g', g,
        offset)], float64 CUDA tensor)."""
        import torch
        cd = np.ascontiguousarray(coupled_dims, dtype=np.int32)
        cg = np.ascontiguousarray(coupled_group, dtype=np.int32)
        gd = np.ascontiguousarray(group_dims, dtype=np.int32)
        if len(cd) != len(cg) or len(proj) != len(cd):
            raise ValueError("one dimension, group and projector per coupled sector")
        ptrs = (ctypes.c_void_p * max(1, len(proj)))()
        for c, pt in enumerate(proj):
            if pt is None:
                if cg[c] >= 0:
                    raise ValueError(f"coupled sector {c} is kept but has no projector")
                continue
            if tuple(pt.shape) != (int(cd[c]), int(gd[cg[c]])):
                raise ValueError(f"projector {c} must be {cd[c]} x {gd[cg[c]]}")
            ptrs[c] = _dev_ptr(pt).value
        basis = Su2Basis(len(cd), _ptr(cd, ctypes.c_int32), _ptr(cg, ctypes.c_int32), len(gd),
                         _ptr(gd, ctypes.c_int32), ptrs)
        b = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
        bo = np.ascontiguousarray(b[:, 0], dtype=np.int32)
        bi = np.ascontiguousarray(b[:, 1], dtype=np.int32)
        boff = np.ascontiguousarray(b[:, 2])
        for k in range(len(b)):  # every block inside the data tensor
            if not (0 <= bo[k] < len(cd) and 0 <= bi[k] < len(cd)):
                raise ValueError(f"block {k}: coupled sector out of range")
            if boff[k] < 0 or boff[k] + int(cd[bo[k]]) * int(cd[bi[k]]) > data.numel():
                raise ValueError(f"block {k} reaches past its data tensor")
        nb, ne = ctypes.c_int32(), ctypes.c_int64()
        self._check(self.lib.dmrg_su2_rotate_size(ctypes.byref(basis), len(b), _ptr(bo, ctypes.c_int32),
                                                  _ptr(bi, ctypes.c_int32), ctypes.byref(nb), ctypes.byref(ne)),
                    None)
        og = np.zeros(max(1, nb.value), dtype=np.int32)
        ig = np.zeros(max(1, nb.value), dtype=np.int32)
        oo = np.zeros(max(1, nb.value), dtype=np.int64)
        out = torch.zeros(max(1, ne.value), dtype=torch.float64, device="cuda")
        self._check(self.lib.dmrg_su2_rotate(self.h, ctypes.byref(basis), len(b), _ptr(bo, ctypes.c_int32),
                                             _ptr(bi, ctypes.c_int32), _ptr(boff, ctypes.c_int64), _dev_ptr(data),
                                             _ptr(og, ctypes.c_int32), _ptr(ig, ctypes.c_int32),
                                             _ptr(oo, ctypes.c_int64), _dev_ptr(out)), self.h)
        return [(int(og[i]), int(ig[i]), int(oo[i])) for i in range(nb.value)], out

    def su2_plan(self, left_sectors, right_sectors, n_elec, two_s, left_ops, right_ops, pairs, precision="fp64"):
        """dmrg_su2_plan_create: a Su2Plan (arguments as in _su2_args;
        precision "fp64" or "bf16x3").  The operator tensors must outlive the
        plan."""
        keep = []
        args = self._su2_args(left_sectors, right_sectors, n_elec, two_s, left_ops, right_ops, pairs, keep)
        h = ctypes.c_void_p()
        self._check(self.lib.dmrg_su2_plan_create(self.h, *args, PRECISIONS[precision], ctypes.byref(h)), self.h)
        return Su2Plan(self, h)

    def debug_diag(self, out):
        self._check(self.lib.dmrg_debug_diag(self.h, _dev_ptr(out)), self.h)
        return out

    def debug_gemm(self, a, b, c, trans_a=False, trans_b=False, alpha=1.0, beta=0,
                   precision="fp64"):
        """c = alpha op(a) op(b) + beta c with the library's GEMM kernel (2-D tensors)."""
        m, n = c.shape
        k = a.shape[0] if trans_a else a.shape[1]
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        st = self.lib.dmrg_debug_gemm(self.h, m, n, k, _dev_ptr(a), a.stride(0), int(trans_a),
                                      _dev_ptr(b), b.stride(0), int(trans_b), _dev_ptr(c),
                                      c.stride(0), float(alpha), int(beta), p)
        self._check(st, self.h)
        return c

    def sigma_info(self, precision="fp64"):
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        info = SigmaInfo()
        self._check(self.lib.dmrg_sigma_get_info(self.h, p, ctypes.byref(info)), self.h)
        return {k: getattr(info, k) for k, _ in SigmaInfo._fields_ if k != "pad"}


class DMRGEnergy:
    """E(h, eri, psi) = psi^T H_eff(h, eri) psi (+ e_core psi^T psi) as a
    torch.autograd.Function of the integrals and the window vector.

    ``DMRGEnergy.apply(h, eri, psi, ctx)``: ctx is a Context whose operators
    were built from these integrals for the window psi belongs to (the MPS
    outside the window is held fixed); dmrg_energy computes E and its psi
    gradient and refuses integrals that differ from the built ones.  The
    backward returns (E_bar * gamma, E_bar * Gamma / 2,
    E_bar * 2 (H_eff psi + e_core psi)) from dmrg_sigma_backward and
    dmrg_energy.
    """

    _fn = None

    @classmethod
    def apply(cls, h, eri, psi, ctx):
        if cls._fn is None:
            import torch

            class _F(torch.autograd.Function):
                @staticmethod
                def forward(fctx, h, eri, psi, c):
                    p = psi.detach().contiguous()
                    grad = torch.empty_like(p)
                    e, _ = c.energy(p, h=h.detach().cpu().numpy(), eri=eri.detach().cpu().numpy(),
                                    grad=grad)
                    fctx.save_for_backward(p, grad)
                    fctx.c = c
                    return torch.tensor(e, dtype=torch.float64, device=psi.device)

                @staticmethod
                def backward(fctx, gE):
                    psi, grad = fctx.saved_tensors
                    dh, deri = fctx.c.sigma_backward(psi)
                    return gE * dh, gE * deri, gE * grad, None

            cls._fn = _F
        return cls._fn.apply(h, eri, psi, ctx)

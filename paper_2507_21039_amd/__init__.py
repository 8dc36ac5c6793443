"""Python binding of libhme.so (include/hme.h): argument marshalling only.

Every step of the |M|^2 computation runs in the library's HIP kernels; PyTorch
supplies device memory and streams.  There is no CPU fallback: if the library
is missing or no GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhme.so")

EEMUMU, GGTT, GGTTG, GGTTGG, GGTTGGG = 0, 1, 2, 3, 4
UUEE, UUEEG, UUEEGG, UUEEGGG = 5, 6, 7, 8  # u ubar -> e+ e- + n g (Drell-Yan family)
FP64, MIXED_FAST, MIXED_PAPER = 0, 1, 2
GAUGE_FD = 0x100  # OR into the precision: internal gluons in the Feynman-diagram gauge
MIXED = MIXED_FAST
PRECISION_NAMES = {FP64: "fp64", MIXED_FAST: "mixed_fast", MIXED_PAPER: "mixed_paper"}
NPAR = {EEMUMU: 4, GGTT: 4, GGTTG: 5, GGTTGG: 6, GGTTGGG: 7, UUEE: 4, UUEEG: 5, UUEEGG: 6, UUEEGGG: 7}
PROCESS_NAMES = {EEMUMU: "e+e- -> mu+mu-", GGTT: "gg -> ttbar", GGTTG: "gg -> ttbar g", GGTTGG: "gg -> ttbar gg",
                 GGTTGGG: "gg -> ttbar ggg", UUEE: "uu~ -> e+e-", UUEEG: "uu~ -> e+e- g", UUEEGG: "uu~ -> e+e- gg",
                 UUEEGGG: "uu~ -> e+e- ggg"}

CUT_NONE, CUT_GLUON_PT, CUT_GLUON_DR, CUT_NO_RETRY = 0, 1, 2, 0x100
GEV2_TO_PB = 0.3893793721e9  # (hbar c)^2 in GeV^2 pb

HME_OK, HME_E_ARG, HME_E_HIP, HME_E_OOM, HME_E_BUDGET, HME_E_TIMEOUT, HME_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6

EXPORTED = ("hme_create", "hme_compute", "hme_query", "hme_good_helicities", "hme_destroy", "hme_last_error",
            "hme_server_create", "hme_submit", "hme_wait", "hme_wait_timed", "hme_server_stats_get",
            "hme_server_destroy", "hme_rambo", "hme_weighted_sum", "hme_compute_select", "hme_compute_alphas",
            "hme_submit_after", "hme_flat_cross_section", "hme_compute_noalloc", "hme_compute_channels")


class SmCard(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("mZ", "wZ", "alpha_inv", "Gf", "mT", "wT")]


class Info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int) for n in ("process", "precision", "npar", "nhel", "ngoodhel", "ncol", "ndiag",
                                            "namp")] + \
               [(n, ctypes.c_double) for n in ("iden", "flops_per_event", "bytes_per_event",
                                               "workspace_bytes_per_event")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "batches", "events", "graphs")] + \
               [("slot_capacity_bytes", ctypes.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class HmeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None


def lib():
    """Load libhme.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_2507_21039_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.hme_create.argtypes = [ctypes.c_int, ctypes.POINTER(SmCard), ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(vp)]
        L.hme_compute.argtypes = [vp, ctypes.c_double, ctypes.c_int64, vp, vp, vp]
        L.hme_compute_noalloc.argtypes = [vp, ctypes.c_double, ctypes.c_int64, vp, vp, vp]
        L.hme_compute_channels.argtypes = [vp, ctypes.c_double, ctypes.c_int64, vp, vp, vp, vp]
        L.hme_query.argtypes = [vp, ctypes.POINTER(Info)]
        L.hme_good_helicities.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
        L.hme_destroy.argtypes = [vp]
        L.hme_last_error.restype = ctypes.c_char_p
        L.hme_server_create.argtypes = [ctypes.POINTER(SmCard), ctypes.c_int, ctypes.c_int, ctypes.c_size_t,
                                        ctypes.c_int, ctypes.POINTER(vp)]
        L.hme_submit.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_int64, vp, vp,
                                 ctypes.POINTER(ctypes.c_uint64)]
        L.hme_submit_after.argtypes = [vp, ctypes.c_int, ctypes.c_double, ctypes.c_int64, vp, vp, vp,
                                       ctypes.POINTER(ctypes.c_uint64)]
        L.hme_flat_cross_section.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_double,
                                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.hme_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double]
        L.hme_wait_timed.argtypes = [vp, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
        L.hme_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
        L.hme_server_destroy.argtypes = [vp]
        L.hme_rambo.argtypes = [ctypes.c_int, ctypes.POINTER(SmCard), ctypes.c_double, ctypes.c_uint64, ctypes.c_int64,
                                ctypes.c_int64, ctypes.c_int, ctypes.c_double, vp, vp, vp]
        L.hme_weighted_sum.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
        L.hme_compute_select.argtypes = [vp, ctypes.c_double, ctypes.c_int64, vp, vp, vp, vp, vp, vp, vp]
        L.hme_compute_alphas.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp]
        for name in ("hme_create", "hme_compute", "hme_query", "hme_good_helicities", "hme_destroy",
                     "hme_server_create", "hme_submit", "hme_wait", "hme_wait_timed", "hme_server_stats_get",
                     "hme_server_destroy", "hme_rambo", "hme_weighted_sum", "hme_compute_select",
                     "hme_compute_alphas", "hme_submit_after", "hme_flat_cross_section", "hme_compute_noalloc",
                     "hme_compute_channels"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def last_error() -> str:
    return lib().hme_last_error().decode()


def _check(rc: int):
    if rc < 0:
        raise HmeError(rc, last_error())
    return rc


def card_struct(card) -> SmCard:
    """card: sequence (mZ, wZ, 1/alpha, G_F, m_top, w_top) or a dict with those keys."""
    if isinstance(card, dict):
        return SmCard(card["mZ"], card["wZ"], card["alpha_inv"], card["Gf"], card["mT"], card["wT"])
    return SmCard(*[float(x) for x in card])


def rambo_ptr(process: int, card, sqrt_s: float, seed: int, first_event: int, nevt: int, cut: int,
              cut_value: float, momenta_ptr: int, weights_ptr: int = 0, stream_ptr: int = 0):
    _check(lib().hme_rambo(process, ctypes.byref(card_struct(card)), float(sqrt_s), int(seed) & 0xFFFFFFFFFFFFFFFF,
                           int(first_event), int(nevt), int(cut), float(cut_value), ctypes.c_void_p(momenta_ptr),
                           ctypes.c_void_p(weights_ptr), ctypes.c_void_p(stream_ptr)))


def _f64_gpu(t, n, what):
    import torch
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"{what} must be a contiguous float64 GPU tensor with at least {n} elements")


def rambo(process: int, card, sqrt_s: float, seed: int, nevt: int, first_event: int = 0, cut: int = CUT_NONE,
          cut_value: float = 0.0, out=None, weights=None, device=None, stream=None):
    """Phase-space points on the GPU (hme_rambo).

    Returns momenta [nevt, npar, 4] (float64, on `device`, default cuda) and, when `weights`
    is True or a tensor, also their phase-space weights [nevt].
    """
    import torch
    dev = torch.device(device) if device is not None else (out.device if out is not None else torch.device("cuda"))
    shape = (int(nevt), NPAR[process], 4)
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=dev)
    _f64_gpu(out, shape[0] * shape[1] * 4, "out")
    want_w = weights is not None and weights is not False
    if weights is True:
        weights = torch.empty(shape[0], dtype=torch.float64, device=out.device)
    if want_w:
        _f64_gpu(weights, shape[0], "weights")
    s = stream if stream is not None else torch.cuda.current_stream(out.device)
    with torch.cuda.device(out.device):
        rambo_ptr(process, card, sqrt_s, seed, first_event, nevt, cut, cut_value, out.data_ptr(),
                  weights.data_ptr() if want_w else 0, s.cuda_stream)
    return (out, weights) if want_w else out


def weighted_sum(me2, weights, stream=None):
    """(sum w |M|^2, sum (w |M|^2)^2) over the events (hme_weighted_sum), as a float64 GPU tensor [2]."""
    import torch
    n = me2.numel()
    _f64_gpu(me2, n, "me2")
    _f64_gpu(weights, n, "weights")
    out = torch.empty(2, dtype=torch.float64, device=me2.device)
    s = stream if stream is not None else torch.cuda.current_stream(me2.device)
    with torch.cuda.device(me2.device):
        _check(lib().hme_weighted_sum(ctypes.c_void_p(me2.data_ptr()), ctypes.c_void_p(weights.data_ptr()), n,
                                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s.cuda_stream)))
    return out


def cross_section_pb(sums, nevt: int, sqrt_s: float):
    """Flat Monte Carlo cross section and its error in pb from weighted_sum's two sums
    (hme_flat_cross_section)."""
    arr = (ctypes.c_double * 2)(float(sums[0]), float(sums[1]))
    sigma, err = ctypes.c_double(), ctypes.c_double()
    _check(lib().hme_flat_cross_section(arr, int(nevt), float(sqrt_s), ctypes.byref(sigma), ctypes.byref(err)))
    return sigma.value, err.value


class Handle:
    """One process on one device (hme_create / hme_compute / hme_destroy)."""

    def __init__(self, process: int, card, precision: int = FP64, device: int = 0):
        self._h = ctypes.c_void_p()
        _check(lib().hme_create(process, ctypes.byref(card_struct(card)), precision, device, ctypes.byref(self._h)))
        self.process, self.precision, self.device = process, precision, device

    def compute_ptr(self, alpha_s: float, nevt: int, momenta_ptr: int, me2_ptr: int, stream_ptr: int = 0):
        _check(lib().hme_compute(self._h, float(alpha_s), int(nevt), ctypes.c_void_p(momenta_ptr),
                                 ctypes.c_void_p(me2_ptr), ctypes.c_void_p(stream_ptr)))

    def compute_noalloc_ptr(self, alpha_s: float, nevt: int, momenta_ptr: int, me2_ptr: int, stream_ptr: int = 0):
        """hme_compute_noalloc: as compute_ptr, with the library's static device scratch."""
        _check(lib().hme_compute_noalloc(self._h, float(alpha_s), int(nevt), ctypes.c_void_p(momenta_ptr),
                                         ctypes.c_void_p(me2_ptr), ctypes.c_void_p(stream_ptr)))

    def compute_channels(self, momenta, alpha_s: float = 0.118, stream=None):
        """|M|^2 and the single-diagram-enhancement channel weights (hme_compute_channels).

        Returns (me2 float64 [nevt], weights float64 [nevt, ndiag]) on the momenta's device.
        """
        import torch
        if momenta.device.type != "cuda" or momenta.dtype != torch.float64 or not momenta.is_contiguous():
            raise ValueError("momenta must be a contiguous float64 GPU tensor")
        if momenta.dim() != 3 or momenta.shape[1] != NPAR[self.process] or momenta.shape[2] != 4:
            raise ValueError(f"momenta must be [nevt, {NPAR[self.process]}, 4]")
        n = momenta.shape[0]
        nd = self.query()["ndiag"]
        me2 = torch.empty(n, dtype=torch.float64, device=momenta.device)
        w = torch.empty((n, nd), dtype=torch.float64, device=momenta.device)
        s = stream if stream is not None else torch.cuda.current_stream(momenta.device)
        _check(lib().hme_compute_channels(self._h, float(alpha_s), n, ctypes.c_void_p(momenta.data_ptr()),
                                          ctypes.c_void_p(me2.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                          ctypes.c_void_p(s.cuda_stream)))
        return me2, w

    def compute(self, momenta, out=None, alpha_s: float = 0.118, stream=None):
        """momenta: torch float64 device tensor [nevt, npar, 4]; returns |M|^2 [nevt] (float64, same device)."""
        import torch
        if momenta.device.type != "cuda" or momenta.dtype != torch.float64 or not momenta.is_contiguous():
            raise ValueError("momenta must be a contiguous float64 GPU tensor")
        if momenta.dim() != 3 or momenta.shape[1] != NPAR[self.process] or momenta.shape[2] != 4:
            raise ValueError(f"momenta must be [nevt, {NPAR[self.process]}, 4]")
        n = momenta.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        if out.dtype != torch.float64 or out.device != momenta.device or out.numel() < n or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor on the momenta's device")
        s = stream if stream is not None else torch.cuda.current_stream(momenta.device)
        self.compute_ptr(alpha_s, n, momenta.data_ptr(), out.data_ptr(), s.cuda_stream)
        return out

    def compute_alphas(self, momenta, alpha_s, out=None, stream=None):
        """|M|^2 with one alpha_s per event (hme_compute_alphas); alpha_s: float64 GPU tensor [nevt]."""
        import torch
        if momenta.device.type != "cuda" or momenta.dtype != torch.float64 or not momenta.is_contiguous():
            raise ValueError("momenta must be a contiguous float64 GPU tensor")
        if momenta.dim() != 3 or momenta.shape[1] != NPAR[self.process] or momenta.shape[2] != 4:
            raise ValueError(f"momenta must be [nevt, {NPAR[self.process]}, 4]")
        n = momenta.shape[0]
        _f64_gpu(alpha_s, n, "alpha_s")
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        _f64_gpu(out, n, "out")
        s = stream if stream is not None else torch.cuda.current_stream(momenta.device)
        _check(lib().hme_compute_alphas(self._h, ctypes.c_void_p(alpha_s.data_ptr()), n,
                                        ctypes.c_void_p(momenta.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        ctypes.c_void_p(s.cuda_stream)))
        return out

    def compute_select(self, momenta, rnd_hel, rnd_col, alpha_s: float = 0.118, stream=None):
        """|M|^2 plus one helicity and one colour flow per event (hme_compute_select).

        rnd_hel, rnd_col: float64 GPU tensors [nevt] of uniforms in [0, 1).
        Returns (me2 float64 [nevt], sel_hel int32 [nevt], sel_col int32 [nevt]).
        """
        import torch
        if momenta.device.type != "cuda" or momenta.dtype != torch.float64 or not momenta.is_contiguous():
            raise ValueError("momenta must be a contiguous float64 GPU tensor")
        if momenta.dim() != 3 or momenta.shape[1] != NPAR[self.process] or momenta.shape[2] != 4:
            raise ValueError(f"momenta must be [nevt, {NPAR[self.process]}, 4]")
        n = momenta.shape[0]
        for t, what in ((rnd_hel, "rnd_hel"), (rnd_col, "rnd_col")):
            _f64_gpu(t, n, what)
            if t.device != momenta.device:
                raise ValueError(f"{what} must be on the momenta's device")
        out = torch.empty(n, dtype=torch.float64, device=momenta.device)
        sh = torch.empty(n, dtype=torch.int32, device=momenta.device)
        sc = torch.empty(n, dtype=torch.int32, device=momenta.device)
        s = stream if stream is not None else torch.cuda.current_stream(momenta.device)
        _check(lib().hme_compute_select(self._h, float(alpha_s), n, ctypes.c_void_p(momenta.data_ptr()),
                                        ctypes.c_void_p(rnd_hel.data_ptr()), ctypes.c_void_p(rnd_col.data_ptr()),
                                        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(sh.data_ptr()),
                                        ctypes.c_void_p(sc.data_ptr()), ctypes.c_void_p(s.cuda_stream)))
        return out, sh, sc

    def query(self) -> dict:
        info = Info()
        _check(lib().hme_query(self._h, ctypes.byref(info)))
        return info.as_dict()

    def good_helicities(self) -> list:
        n = _check(lib().hme_good_helicities(self._h, None, 0))
        buf = (ctypes.c_int * max(n, 1))()
        _check(lib().hme_good_helicities(self._h, buf, n))
        return list(buf[:n])

    def close(self):
        if self._h:
            _check(lib().hme_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Server:
    """Persistent request loop over all processes on one device (hme_server_*)."""

    def __init__(self, card, precision: int = FP64, device: int = 0, hbm_budget_bytes: int = 1 << 30,
                 nstreams: int = 4):
        self._s = ctypes.c_void_p()
        _check(lib().hme_server_create(ctypes.byref(card_struct(card)), precision, device, int(hbm_budget_bytes),
                                       nstreams, ctypes.byref(self._s)))

    def submit_ptr(self, process: int, alpha_s: float, nevt: int, momenta_ptr: int, me2_ptr: int) -> int:
        rid = ctypes.c_uint64()
        _check(lib().hme_submit(self._s, process, float(alpha_s), int(nevt), ctypes.c_void_p(momenta_ptr),
                                ctypes.c_void_p(me2_ptr), ctypes.byref(rid)))
        return rid.value

    def submit_after_ptr(self, process: int, alpha_s: float, nevt: int, momenta_ptr: int, me2_ptr: int,
                         stream_ptr: int) -> int:
        rid = ctypes.c_uint64()
        _check(lib().hme_submit_after(self._s, process, float(alpha_s), int(nevt), ctypes.c_void_p(momenta_ptr),
                                      ctypes.c_void_p(me2_ptr), ctypes.c_void_p(stream_ptr), ctypes.byref(rid)))
        return rid.value

    def submit(self, process: int, momenta, out, alpha_s: float = 0.118, stream=None) -> int:
        """momenta [nevt, npar, 4] float64 GPU tensor, out [nevt] float64 GPU tensor (kept alive by the caller).
        The request reads the momenta after the work queued so far on `stream` (default: torch's current
        stream), so they may still be in flight there (hme_submit_after)."""
        import torch
        if momenta.dim() != 3 or momenta.shape[1] != NPAR[process] or not momenta.is_contiguous():
            raise ValueError(f"momenta must be contiguous [nevt, {NPAR[process]}, 4]")
        if out.numel() < momenta.shape[0] or not out.is_contiguous():
            raise ValueError("out too small or not contiguous")
        s = stream if stream is not None else torch.cuda.current_stream(momenta.device)
        return self.submit_after_ptr(process, alpha_s, momenta.shape[0], momenta.data_ptr(), out.data_ptr(),
                                     s.cuda_stream)

    def wait(self, req_id: int, timeout_s: float = -1.0):
        """Returns the request's submit-to-completion latency in seconds, or None on timeout."""
        lat = ctypes.c_double()
        rc = lib().hme_wait_timed(self._s, req_id, float(timeout_s), ctypes.byref(lat))
        if rc == HME_E_TIMEOUT:
            return None
        _check(rc)
        return lat.value

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().hme_server_stats_get(self._s, ctypes.byref(st)))
        return st.as_dict()

    def close(self):
        if self._s:
            _check(lib().hme_server_destroy(self._s))
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

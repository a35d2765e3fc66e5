"""ctypes binding of libbse.so: the C entry points under the same names.

Argument marshalling only.  Pointers are passed as integers (device
addresses, e.g. `tensor.data_ptr()`), streams as the raw hipStream_t value.
The library must be built (`python -m paper_1904_05575_amd.build`); there is
no fallback.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libbse.so")

BSE_TDA, BSE_FULL = 0, 1
BSE_SINGLET, BSE_TRIPLET, BSE_RPA, BSE_IP = 0, 1, 2, 3
BSE_PREC_FP64, BSE_PREC_FP32, BSE_PREC_BF16X3 = 0, 1, 2
BSE_STAGE_BUILD, BSE_STAGE_SOLVE = 0, 1
STATUS = {0: "BSE_OK", 1: "BSE_ERR_ARG", 2: "BSE_ERR_WORKSPACE", 3: "BSE_ERR_HIP"}
EXPORTS = ("bse_workspace_size", "bse_build", "bse_solve", "bse_oscillator", "bse_spectrum",
           "bse_transitions", "bse_dielectric_tensor", "bse_loss", "bse_screening_workspace_size",
           "bse_screening", "bse_status_string", "bse_timing_enable", "bse_timing_report",
           "bse_batch_workspace_size", "bse_batch_create", "bse_batch_capture", "bse_batch_run",
           "bse_batch_destroy", "bse_tune_set", "bse_tune_get", "bse_solve_noalloc", "bse_pair_elements")
NOALLOC_SCRATCH_BYTES = 32 << 20  # BSE_NOALLOC_SCRATCH_BYTES of bse.h
TUNE_SITES = {"hemv_unit": 0, "gemm_squared": 1, "gemm_potrf": 2, "gemm_her2k": 3,
              "gemm_stage2": 4, "gemm_exchange": 5, "direct": 6, "gemm_products": 7,
              "batch_sweep": 8, "gemm_vectors": 9,
              "batch_align": 10, "gemm_squared_s": 11}


class BseDesc(ctypes.Structure):
    _fields_ = [("nk", ctypes.c_int32), ("nv", ctypes.c_int32), ("nc", ctypes.c_int32),
                ("ng", ctypes.c_int32), ("coupling", ctypes.c_int32), ("type", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("split_terms", ctypes.c_int32),
                ("kappa", ctypes.c_double), ("scissor", ctypes.c_double),
                ("ld", ctypes.c_int64)]


class BseInputs(ctypes.Structure):
    _fields_ = [("eps_v", ctypes.c_void_p), ("eps_c", ctypes.c_void_p),
                ("Mcv", ctypes.c_void_p), ("Mvv", ctypes.c_void_p), ("Mcc", ctypes.c_void_p),
                ("Ncv", ctypes.c_void_p), ("Nvc", ctypes.c_void_p), ("W", ctypes.c_void_p),
                ("vbar", ctypes.c_void_p), ("qmap", ctypes.c_void_p), ("qramap", ctypes.c_void_p),
                ("nq", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("mcc_env", ctypes.c_void_p), ("mcc_key", ctypes.c_uint64)]


class BseOrbDesc(ctypes.Structure):
    _fields_ = [("nk", ctypes.c_int32), ("nv", ctypes.c_int32), ("nc", ctypes.c_int32),
                ("ng", ctypes.c_int32), ("nkb", ctypes.c_int32), ("coupling", ctypes.c_int32)]


class BseScreenDesc(ctypes.Structure):
    _fields_ = [("nk", ctypes.c_int32), ("nv", ctypes.c_int32), ("nc", ctypes.c_int32),
                ("ng", ctypes.c_int32), ("inv_vc", ctypes.c_double),
                ("units_per_hartree", ctypes.c_double)]


class BseTuneEntry(ctypes.Structure):
    _fields_ = [("site", ctypes.c_int32), ("size_max", ctypes.c_int32),
                ("choice", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class BseError(RuntimeError):
    pass


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise BseError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1904_05575_amd.build`")
        # PyTorch ships its own HIP and HSA runtimes under the same sonames as
        # the system's.  Loaded after them, this library binds to torch's copy;
        # loaded first, it would bind the system's and torch would then load a
        # second runtime, in which case this library's launches find no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_double, ctypes.c_size_t)
        L.bse_workspace_size.argtypes = [ctypes.POINTER(BseDesc), i32]
        L.bse_workspace_size.restype = sz
        L.bse_build.argtypes = [ctypes.POINTER(BseDesc), ctypes.POINTER(BseInputs), vp, vp, vp, sz,
                                vp, vp]
        L.bse_build.restype = ctypes.c_int
        L.bse_solve.argtypes = [ctypes.POINTER(BseDesc), vp, vp, vp, vp, vp, i64, vp, vp, vp, sz,
                                vp, vp]
        L.bse_solve.restype = ctypes.c_int
        L.bse_solve_noalloc.argtypes = [ctypes.POINTER(BseDesc), vp, vp, vp, vp, vp, i64, vp, vp,
                                        vp, vp]
        L.bse_solve_noalloc.restype = ctypes.c_int
        L.bse_pair_elements.argtypes = [ctypes.POINTER(BseOrbDesc), vp, vp, vp, vp, vp, vp, vp,
                                        vp, vp]
        L.bse_pair_elements.restype = ctypes.c_int
        L.bse_coulomb.argtypes = [i32, vp, dbl, ctypes.POINTER(dbl), vp, vp, vp]
        L.bse_coulomb.restype = ctypes.c_int
        L.bse_probe.argtypes = [i64, i32, vp, vp, vp, vp]
        L.bse_probe.restype = ctypes.c_int
        L.bse_oscillator.argtypes = [i64, vp, i64, vp, vp, vp]
        L.bse_oscillator.restype = ctypes.c_int
        L.bse_spectrum.argtypes = [i64, vp, vp, dbl, dbl, i64, vp, vp, vp]
        L.bse_spectrum.restype = ctypes.c_int
        L.bse_transitions.argtypes = [i64, vp, i64, i32, vp, i64, vp, i64, vp]
        L.bse_transitions.restype = ctypes.c_int
        L.bse_dielectric_tensor.argtypes = [i64, vp, i32, vp, i64, dbl, dbl, i64, vp, vp, vp]
        L.bse_dielectric_tensor.restype = ctypes.c_int
        L.bse_loss.argtypes = [i64, vp, i64, dbl, vp, vp, vp]
        L.bse_loss.restype = ctypes.c_int
        L.bse_screening_workspace_size.argtypes = [ctypes.POINTER(BseScreenDesc)]
        L.bse_screening_workspace_size.restype = sz
        L.bse_screening.argtypes = [ctypes.POINTER(BseScreenDesc), vp, vp, vp, vp, vp, vp, vp, vp,
                                    sz, vp, vp]
        L.bse_screening.restype = ctypes.c_int
        L.bse_timing_enable.argtypes = [i32, ctypes.c_char_p]
        L.bse_timing_enable.restype = None
        L.bse_timing_report.argtypes = [ctypes.c_char_p, i64]
        L.bse_timing_report.restype = i64
        L.bse_batch_workspace_size.argtypes = [i32, ctypes.POINTER(BseDesc), i32]
        L.bse_batch_workspace_size.restype = sz
        L.bse_batch_create.argtypes = [i32, ctypes.POINTER(BseDesc), i32, ctypes.POINTER(vp)]
        L.bse_batch_create.restype = ctypes.c_int
        P = ctypes.POINTER(vp)
        L.bse_batch_capture.argtypes = [vp, ctypes.POINTER(BseInputs), P, P, P, P, P,
                                        ctypes.POINTER(dbl), ctypes.POINTER(dbl),
                                        ctypes.POINTER(i64), P, P, vp, sz, vp, vp]
        L.bse_batch_capture.restype = ctypes.c_int
        L.bse_batch_run.argtypes = [vp, vp]
        L.bse_batch_run.restype = ctypes.c_int
        L.bse_batch_destroy.argtypes = [vp]
        L.bse_batch_destroy.restype = None
        L.bse_tune_set.argtypes = [ctypes.POINTER(BseTuneEntry), i32]
        L.bse_tune_set.restype = ctypes.c_int
        L.bse_tune_get.argtypes = [ctypes.POINTER(BseTuneEntry), i32]
        L.bse_tune_get.restype = i32
        L.bse_status_string.argtypes = [ctypes.c_int]
        L.bse_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status: int, what: str) -> None:
    if status != 0:
        msg = lib().bse_status_string(status).decode()
        raise BseError(f"{what}: {STATUS.get(status, status)} ({msg})")


def bse_workspace_size(desc: BseDesc, stage: int) -> int:
    return int(lib().bse_workspace_size(ctypes.byref(desc), stage))


def bse_build(desc: BseDesc, inputs: BseInputs, H0: int, H1: int, ws: int, ws_bytes: int,
              info: int, stream: int) -> None:
    _check(lib().bse_build(ctypes.byref(desc), ctypes.byref(inputs), H0, H1 or None, ws, ws_bytes,
                           info, stream or None), "bse_build")


def bse_solve(desc: BseDesc, H0: int, H1: int, E: int, XpY: int, XmY: int, ldx: int, probe: int,
              osc: int, ws: int, ws_bytes: int, info: int, stream: int) -> None:
    _check(lib().bse_solve(ctypes.byref(desc), H0, H1 or None, E, XpY or None, XmY or None, ldx,
                           probe or None, osc or None, ws, ws_bytes, info, stream or None),
           "bse_solve")


def bse_solve_noalloc(desc: BseDesc, H0: int, H1: int, E: int, XpY: int, XmY: int, ldx: int,
                      probe: int, osc: int, info: int, stream: int) -> None:
    _check(lib().bse_solve_noalloc(ctypes.byref(desc), H0, H1 or None, E, XpY or None,
                                   XmY or None, ldx, probe or None, osc or None, info,
                                   stream or None), "bse_solve_noalloc")


def bse_pair_elements(desc: BseOrbDesc, C: int, kpg: int, mkg: int, Mcv: int, Mvv: int,
                      Mcc: int, Ncv: int, Nvc: int, stream: int) -> None:
    _check(lib().bse_pair_elements(ctypes.byref(desc), C, kpg, mkg or None, Mcv, Mvv, Mcc,
                                   Ncv or None, Nvc or None, stream or None),
           "bse_pair_elements")


def bse_coulomb(ng: int, gvec: int, alat: float, Q, vbar: int, gq: int, stream: int) -> None:
    q = (ctypes.c_double * 3)(*[float(x) for x in Q])
    _check(lib().bse_coulomb(ng, gvec, alat, q, vbar, gq, stream or None), "bse_coulomb")


def bse_probe(n: int, ng: int, Mcv: int, gq: int, probe: int, stream: int) -> None:
    _check(lib().bse_probe(n, ng, Mcv, gq, probe, stream or None), "bse_probe")


def bse_oscillator(n: int, XpY: int, ldx: int, probe: int, osc: int, stream: int) -> None:
    _check(lib().bse_oscillator(n, XpY, ldx, probe, osc, stream or None), "bse_oscillator")


def bse_spectrum(n: int, E: int, osc: int, pref: float, eta: float, nw: int, omega: int, eps: int,
                 stream: int) -> None:
    _check(lib().bse_spectrum(n, E, osc, pref, eta, nw, omega, eps, stream or None),
           "bse_spectrum")


def bse_transitions(n: int, XpY: int, ldx: int, nprobe: int, probe: int, ldp: int, t: int,
                    ldt: int, stream: int) -> None:
    _check(lib().bse_transitions(n, XpY or None, ldx, nprobe, probe or None, ldp, t or None, ldt,
                                 stream or None), "bse_transitions")


def bse_dielectric_tensor(n: int, E: int, nd: int, t: int, ldt: int, pref: float, eta: float,
                          nw: int, omega: int, eps: int, stream: int) -> None:
    _check(lib().bse_dielectric_tensor(n, E or None, nd, t or None, ldt, pref, eta, nw,
                                       omega or None, eps or None, stream or None),
           "bse_dielectric_tensor")


def bse_loss(nw: int, eps: int, inc: int, vinv: float, loss: int, sqw: int, stream: int) -> None:
    _check(lib().bse_loss(nw, eps or None, inc, vinv, loss or None, sqw or None, stream or None),
           "bse_loss")


def bse_screening_workspace_size(desc: BseScreenDesc) -> int:
    return int(lib().bse_screening_workspace_size(ctypes.byref(desc)))


def bse_screening(desc: BseScreenDesc, eps_v: int, eps_c: int, kqmap: int, Svc: int, Scv: int,
                  vsqrt: int, W: int, ws: int, ws_bytes: int, info: int, stream: int) -> None:
    _check(lib().bse_screening(ctypes.byref(desc), eps_v or None, eps_c or None, kqmap or None,
                               Svc or None, Scv or None, vsqrt or None, W or None, ws or None,
                               ws_bytes, info or None, stream or None), "bse_screening")


def bse_timing_enable(on: bool, name: str | None = None) -> None:
    lib().bse_timing_enable(1 if on else 0, name.encode() if name else None)


def bse_timing_report() -> dict:
    """{kernel name: (launches, total ms)} since the last report."""
    n = lib().bse_timing_report(None, 0)
    buf = ctypes.create_string_buffer(int(n) + 1)
    lib().bse_timing_report(buf, n + 1)
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


def _ptrs(vals):
    arr = (ctypes.c_void_p * len(vals))(*[v or None for v in vals])
    return ctypes.cast(arr, ctypes.POINTER(ctypes.c_void_p)), arr


def bse_batch_workspace_size(descs, nbranch: int) -> int:
    arr = (BseDesc * len(descs))(*descs)
    return int(lib().bse_batch_workspace_size(len(descs), arr, nbranch))


def bse_batch_create(descs, nbranch: int) -> int:
    arr = (BseDesc * len(descs))(*descs)
    h = ctypes.c_void_p()
    _check(lib().bse_batch_create(len(descs), arr, nbranch, ctypes.byref(h)), "bse_batch_create")
    return h.value


def bse_batch_capture(batch: int, inputs, H0, H1, E, probe, osc, pref, eta, nw, omega, eps,
                      ws: int, ws_bytes: int, info: int, stream: int) -> None:
    n = len(inputs)
    inarr = (BseInputs * n)(*inputs)
    keep = [_ptrs(v) for v in (H0, H1, E, probe, osc, omega, eps)]
    dbl = ctypes.c_double * n
    _check(lib().bse_batch_capture(batch, inarr, keep[0][0], keep[1][0], keep[2][0], keep[3][0],
                                   keep[4][0], dbl(*pref), dbl(*eta), (ctypes.c_int64 * n)(*nw),
                                   keep[5][0], keep[6][0], ws, ws_bytes, info, stream or None),
           "bse_batch_capture")


def bse_batch_run(batch: int, stream: int) -> None:
    _check(lib().bse_batch_run(batch, stream or None), "bse_batch_run")


def bse_batch_destroy(batch: int) -> None:
    lib().bse_batch_destroy(batch)


def bse_tune_set(entries) -> None:
    """entries: iterable of (site, size_max, choice); an empty list clears the table."""
    entries = list(entries)
    arr = (BseTuneEntry * max(1, len(entries)))(*[BseTuneEntry(s, m, c, 0) for s, m, c in entries])
    _check(lib().bse_tune_set(arr, len(entries)), "bse_tune_set")


def bse_tune_get() -> list:
    n = int(lib().bse_tune_get(None, 0))
    arr = (BseTuneEntry * max(1, n))()
    lib().bse_tune_get(arr, n)
    return [(arr[i].site, arr[i].size_max, arr[i].choice) for i in range(n)]

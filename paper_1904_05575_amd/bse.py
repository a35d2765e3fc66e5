"""Host-side driver of the BSE library: device buffers, descriptor, calls.

PyTorch supplies device memory and the stream; every step of the method runs
in libbse.so.  The small host computations here are scalars of the problem's geometry
(the kernel prefactor 1/V_c of eq. vft, v(Q) of the spectrum's prefactor) and
the probe vectors conj(D) of eq. tlambdai; the Coulomb potential of eq.
vbar_def and the probe of eq. osci are formed by the library.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L

HARTREE_EV = 27.211386245988
TYPES = {"singlet": L.BSE_SINGLET, "triplet": L.BSE_TRIPLET, "rpa": L.BSE_RPA, "ip": L.BSE_IP}
PRECISIONS = {"fp64": (L.BSE_PREC_FP64, 0), "fp32": (L.BSE_PREC_FP32, 0),
              "bf16x6": (L.BSE_PREC_BF16X3, 6), "bf16x3": (L.BSE_PREC_BF16X3, 3)}


def device_vbar_probe(gvec: np.ndarray, alat: float, q, n: int, ng: int, Mcv: torch.Tensor,
                      device) -> tuple[torch.Tensor, torch.Tensor]:
    """The exchange term's vbar (eq. vbar_def) and the probe conj(M(G_Q)) of eq.
    osci, formed by the library (bse_coulomb, bse_probe) on the current stream."""
    g = np.ascontiguousarray(gvec, dtype=np.int32)
    if g.shape != (ng, 3):
        raise ValueError(f"gvec has shape {g.shape}, expected ({ng}, 3)")
    gd = _dev(g, torch.int32, device)
    vbar = torch.empty(ng, dtype=torch.float64, device=device)
    gq = torch.zeros(1, dtype=torch.int32, device=device)
    probe = torch.empty(n, dtype=torch.complex128, device=device)
    s = torch.cuda.current_stream().cuda_stream
    L.bse_coulomb(ng, gd.data_ptr(), float(alat), q, vbar.data_ptr(), gq.data_ptr(), s)
    L.bse_probe(n, ng, Mcv.data_ptr(), gq.data_ptr(), probe.data_ptr(), s)
    return vbar, probe


def coulomb_v0(q) -> float:
    """4 pi / |Q|^2, with |Q|^2 taken as 0.01 bohr^-2 at Q = 0."""
    q2 = float(np.dot(q, q))
    return 4.0 * np.pi / (q2 if q2 > 1e-12 else 0.01)


def kernel_prefactor(kernel_scale: float, nk: int, cell_volume: float) -> float:
    """s * Ha / (Nk * Omega): 1/V_c in eV for lengths in bohr."""
    return kernel_scale * HARTREE_EV / (nk * cell_volume)


def _dev(a: np.ndarray, dtype, device) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype)


def sphere_partners(kvec: np.ndarray, gvec: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """int32 [NK][NG] tables of bse_pair_elements: position in the orbital
    sphere of K + G and of -K - G, -1 outside.  Integer vectors are keyed by
    one integer (each coordinate offset into [0, 2^20)) and searched in the
    sorted keys of the sphere."""
    def key(v):
        v = np.asarray(v, dtype=np.int64) + (1 << 19)
        return (v[..., 0] << 40) | (v[..., 1] << 20) | v[..., 2]
    ks = key(kvec)
    order = np.argsort(ks)
    sk = ks[order]

    def find(vecs):
        q = key(vecs)
        at = np.clip(np.searchsorted(sk, q), 0, len(sk) - 1)
        return np.where(sk[at] == q, order[at], -1).astype(np.int32)
    plus = find(kvec[:, None, :] + gvec[None, :, :])
    minus = find(-kvec[:, None, :] - gvec[None, :, :])
    return plus, minus


class Problem:
    """One BSE problem resident on the GPU."""

    def __init__(self, inputs: dict, bse_type: str = "singlet", device: str = "cuda",
                 precision: str = "fp64"):
        from . import tune
        tune.load()  # the autotuner's tile choices, when a table is present
        w = inputs["workload"]
        self.workload = w
        self.device = torch.device(device)
        self.nk, self.nv, self.nc, self.ng = w.nk, w.nv, w.nc, w.ng
        self.n = w.nk * w.nv * w.nc
        self.full = w.coupling == "full"
        c128, f64 = torch.complex128, torch.float64
        dv = self.device
        self.t = {
            "eps_v": _dev(inputs["eps_v"], f64, dv),
            "eps_c": _dev(inputs["eps_c"], f64, dv),
            "W": _dev(inputs["W"], c128, dv),
            "qmap": _dev(inputs["qmap"], torch.int32, dv),
        }
        if self.full:
            self.t["qramap"] = _dev(inputs["qramap"], torch.int32, dv)
        if inputs.get("C") is not None:
            # pair elements formed on the device from the orbitals
            self.form_pair_elements(inputs)
        else:
            self.t["Mcv"] = _dev(inputs["Mcv"], c128, dv)
            self.t["Mvv"] = _dev(inputs["Mvv"], c128, dv)
            if inputs.get("Mcc") is not None:
                self.t["Mcc"] = _dev(inputs["Mcc"], c128, dv)
            else:  # drawn in place from an envelope and a key
                self.t["mcc_env"] = _dev(inputs["mcc_env"], f64, dv)
            if self.full:
                self.t["Ncv"] = _dev(inputs["Ncv"], c128, dv)
                self.t["Nvc"] = _dev(inputs["Nvc"], c128, dv)
        self.t["vbar"], self.t["probe"] = device_vbar_probe(
            inputs["gvec"], inputs["alat"], w.q, self.n, w.ng, self.t["Mcv"], dv)
        self.t["omega"] = _dev(inputs["omega"], f64, dv)
        if inputs.get("Dcv") is not None:  # column i = conj(D_{., i}), column-major n x 3
            self.t["dprobe"] = _dev(np.conj(inputs["Dcv"]).T, c128, dv)
        self.kappa = kernel_prefactor(w.kernel_scale, w.nk, inputs["cell_volume"])
        self.pref = 2.0 * self.kappa * coulomb_v0(w.q)
        self.tensor_pref = 8.0 * np.pi * self.kappa  # spin 2, 1/V_c, 4 pi of v(q) (eq. mofd)
        self.vinv = 1.0 / coulomb_v0(w.q)
        self.eta = w.eta
        self.desc = L.BseDesc(nk=w.nk, nv=w.nv, nc=w.nc, ng=w.ng,
                              coupling=L.BSE_FULL if self.full else L.BSE_TDA,
                              type=TYPES[bse_type], prec=PRECISIONS[precision][0],
                              split_terms=PRECISIONS[precision][1],
                              kappa=self.kappa, scissor=w.scissor, ld=self.n)
        p = lambda k: self.t[k].data_ptr() if k in self.t else None  # noqa: E731
        self.inp = L.BseInputs(eps_v=p("eps_v"), eps_c=p("eps_c"), Mcv=p("Mcv"), Mvv=p("Mvv"),
                               Mcc=p("Mcc"), Ncv=p("Ncv"), Nvc=p("Nvc"), W=p("W"),
                               vbar=p("vbar"), qmap=p("qmap"), qramap=p("qramap"),
                               nq=int(inputs["W"].shape[0]), reserved=0,
                               mcc_env=p("mcc_env"), mcc_key=int(inputs.get("mcc_key", 0)))
        self.info = torch.zeros(1, dtype=torch.int32, device=dv)
        self.ws_build = torch.empty(max(1, L.bse_workspace_size(self.desc, L.BSE_STAGE_BUILD)),
                                    dtype=torch.uint8, device=dv)
        self.ws_solve = torch.empty(max(1, L.bse_workspace_size(self.desc, L.BSE_STAGE_SOLVE)),
                                    dtype=torch.uint8, device=dv)

    def form_pair_elements(self, inputs: dict) -> None:
        """Mcv, Mvv, Mcc (Ncv, Nvc) on the device from the orbital coefficients
        (bse_pair_elements); sets self.t and keeps C and the partner tables."""
        w = inputs["workload"]
        dv, c128 = self.device, torch.complex128
        P = w.nk * (w.nk + 1) // 2
        plus, minus = sphere_partners(inputs["kvec"], inputs["gvec"])
        t = self.t
        t["C"] = _dev(inputs["C"], c128, dv)
        t["kpg"] = _dev(plus, torch.int32, dv)
        t["mkg"] = _dev(minus, torch.int32, dv)
        t["Mcv"] = torch.empty((self.n, w.ng), dtype=c128, device=dv)
        t["Mvv"] = torch.empty((P, w.nv, w.nv, w.ng), dtype=c128, device=dv)
        t["Mcc"] = torch.empty((P, w.nc, w.nc, w.ng), dtype=c128, device=dv)
        if self.full:
            t["Ncv"] = torch.empty((P, w.nc, w.nv, w.ng), dtype=c128, device=dv)
            t["Nvc"] = torch.empty((P, w.nv, w.nc, w.ng), dtype=c128, device=dv)
        self.orb_desc = L.BseOrbDesc(nk=w.nk, nv=w.nv, nc=w.nc, ng=w.ng, nkb=w.orbitals,
                                     coupling=L.BSE_FULL if self.full else L.BSE_TDA)
        self.pair_elements()

    def pair_elements(self) -> None:
        """Form the pair elements again from the resident orbitals (enqueued)."""
        t = self.t
        p = lambda k: t[k].data_ptr() if k in t else 0  # noqa: E731
        L.bse_pair_elements(self.orb_desc, p("C"), p("kpg"), p("mkg"), p("Mcv"), p("Mvv"),
                            p("Mcc"), p("Ncv"), p("Nvc"), self.stream())

    def set_precision(self, precision: str) -> None:
        """Switch the arithmetic of the assembly (same inputs and workspaces)."""
        self.desc.prec, self.desc.split_terms = PRECISIONS[precision]

    @staticmethod
    def stream() -> int:
        return torch.cuda.current_stream().cuda_stream

    def check_info(self) -> None:
        torch.cuda.synchronize()
        code = int(self.info.item())
        if code != 0:
            raise L.BseError(f"device status info = {code}")

    def alloc_matrices(self):
        n = self.n
        H0 = torch.empty((n, n), dtype=torch.complex128, device=self.device)
        H1 = torch.empty((n, n), dtype=torch.complex128, device=self.device) if self.full else None
        return H0, H1

    def reset_info(self) -> None:
        """Clear the device status word (a fill kernel on the current stream).
        The library's kernels return at entry while it is non-zero, so every
        build starts from a cleared word: a failure of an earlier call does
        not silence the next one."""
        self.info.zero_()

    def build(self, H0=None, H1=None):
        """A+B and A-B (full) or A (TDA), column-major: element (i, j) is H.T[i, j].
        Clears the status word first (see reset_info)."""
        if H0 is None:
            H0, H1 = self.alloc_matrices()
        self.reset_info()
        L.bse_build(self.desc, self.inp, H0.data_ptr(), H1.data_ptr() if H1 is not None else 0,
                    self.ws_build.data_ptr(), self.ws_build.numel(), self.info.data_ptr(),
                    self.stream())
        return H0, H1

    def solve(self, H0, H1, vectors: bool = False, probe: bool = True, xmy: bool = False):
        """(E, X+Y, |t|^2); with xmy=True (implies vectors) (E, X+Y, X-Y, |t|^2).
        X+Y and X-Y are column-major n x n: column l is X.T[l]."""
        n = self.n
        vectors = vectors or xmy
        E = torch.empty(n, dtype=torch.float64, device=self.device)
        XpY = torch.empty((n, n), dtype=torch.complex128, device=self.device) if vectors else None
        XmY = torch.empty((n, n), dtype=torch.complex128, device=self.device) if xmy else None
        osc = torch.empty(n, dtype=torch.float64, device=self.device) if probe else None
        L.bse_solve(self.desc, H0.data_ptr(), H1.data_ptr() if H1 is not None else 0,
                    E.data_ptr(), XpY.data_ptr() if XpY is not None else 0,
                    XmY.data_ptr() if XmY is not None else 0, n,
                    self.t["probe"].data_ptr() if probe else 0,
                    osc.data_ptr() if osc is not None else 0, self.ws_solve.data_ptr(),
                    self.ws_solve.numel(), self.info.data_ptr(), self.stream())
        if xmy:
            return E, XpY, XmY, osc
        return E, XpY, osc

    def spectrum(self, E, osc):
        nw = self.t["omega"].numel()
        eps = torch.empty(nw, dtype=torch.complex128, device=self.device)
        L.bse_spectrum(self.n, E.data_ptr(), osc.data_ptr(), self.pref, self.eta, nw,
                       self.t["omega"].data_ptr(), eps.data_ptr(), self.stream())
        return eps

    def oscillator(self, XpY):
        osc = torch.empty(self.n, dtype=torch.float64, device=self.device)
        L.bse_oscillator(self.n, XpY.data_ptr(), self.n, self.t["probe"].data_ptr(),
                         osc.data_ptr(), self.stream())
        return osc

    def transitions(self, XpY, probes=None):
        """t (column-major n x nprobe, as a [nprobe, n] tensor) of eq. tlambdai
        for the probe columns conj(D) (default: the three Cartesian directions)."""
        P = self.t["dprobe"] if probes is None else probes
        nprobe = P.shape[0]
        t = torch.empty((nprobe, self.n), dtype=torch.complex128, device=self.device)
        L.bse_transitions(self.n, XpY.data_ptr(), self.n, nprobe, P.data_ptr(), self.n,
                          t.data_ptr(), self.n, self.stream())
        return t

    def dielectric_tensor(self, E, t):
        """eps[w, a, b] of eq. epsmij from bse_transitions' t ([nd, n])."""
        nd, nw = t.shape[0], self.t["omega"].numel()
        eps = torch.empty((nw, nd, nd), dtype=torch.complex128, device=self.device)
        L.bse_dielectric_tensor(self.n, E.data_ptr(), nd, t.data_ptr(), self.n, self.tensor_pref,
                                self.eta, nw, self.t["omega"].data_ptr(), eps.data_ptr(),
                                self.stream())
        return eps

    def loss(self, eps, diag: int | None = None):
        """(-Im 1/eps, S(Q, w)) for a scalar spectrum [nw], or for the diagonal
        element (diag, diag) of a tensor [nw, nd, nd]."""
        nw = eps.shape[0]
        ptr, inc = eps.data_ptr(), 1
        if diag is not None:
            nd = eps.shape[1]
            ptr += 16 * diag * (nd + 1)
            inc = nd * nd
        L_ = torch.empty(nw, dtype=torch.float64, device=self.device)
        S = torch.empty(nw, dtype=torch.float64, device=self.device)
        L.bse_loss(nw, ptr, inc, self.vinv, L_.data_ptr(), S.data_ptr(), self.stream())
        return L_, S

    def run(self, vectors: bool = False):
        """build -> solve -> spectrum; returns host arrays."""
        H0, H1 = self.build()
        E, XpY, osc = self.solve(H0, H1, vectors=vectors)
        eps = self.spectrum(E, osc)
        self.check_info()
        out = {"E": E.cpu().numpy(), "osc": osc.cpu().numpy(), "eps": eps.cpu().numpy()}
        if vectors:
            out["XpY"] = XpY.T.cpu().numpy()  # column-major storage -> [a, l]
        return out


class Screening:
    """The static RPA screening of one k-mesh resident on the GPU: W(q) for
    every q of the mesh (bse_screening), in the layout bse_build takes."""

    def __init__(self, sinputs: dict, device: str = "cuda"):
        w = sinputs["workload"]
        self.workload = w
        self.device = torch.device(device)
        dv, c128, f64 = self.device, torch.complex128, torch.float64
        self.nk, self.ng = w.nk, w.ng
        G = sinputs["gvec"].astype(np.float64) * (2.0 * np.pi / sinputs["alat"])
        p2 = np.sum((sinputs["qcart"][:, None, :] + G[None, :, :]) ** 2, axis=2)
        vsqrt = np.sqrt(4.0 * np.pi / np.where(p2 < 1e-12, 0.01, p2))  # v(q+G)^1/2
        self.t = {"eps_v": _dev(sinputs["eps_v"], f64, dv), "eps_c": _dev(sinputs["eps_c"], f64, dv),
                  "kqmap": _dev(sinputs["kqmap"], torch.int32, dv),
                  "Svc": _dev(sinputs["Svc"], c128, dv), "Scv": _dev(sinputs["Scv"], c128, dv),
                  "vsqrt": _dev(vsqrt, f64, dv)}
        self.desc = L.BseScreenDesc(nk=w.nk, nv=w.nv, nc=w.nc, ng=w.ng,
                                    inv_vc=1.0 / (w.nk * sinputs["cell_volume"]),
                                    units_per_hartree=HARTREE_EV)
        self.ws = torch.empty(max(1, L.bse_screening_workspace_size(self.desc)),
                              dtype=torch.uint8, device=dv)
        self.info = torch.zeros(1, dtype=torch.int32, device=dv)

    def run(self, W=None):
        """W[q, G, G'] (complex128 tensor on the device)."""
        if W is None:
            W = torch.empty((self.nk, self.ng, self.ng), dtype=torch.complex128, device=self.device)
        t = self.t
        L.bse_screening(self.desc, t["eps_v"].data_ptr(), t["eps_c"].data_ptr(),
                        t["kqmap"].data_ptr(), t["Svc"].data_ptr(), t["Scv"].data_ptr(),
                        t["vsqrt"].data_ptr(), W.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
                        self.info.data_ptr(), torch.cuda.current_stream().cuda_stream)
        return W

    def check_info(self) -> None:
        torch.cuda.synchronize()
        code = int(self.info.item())
        if code != 0:
            raise L.BseError(f"device status info = {code}")


"""Batched BSE problems (one per momentum transfer Q) replayed as one HIP
graph: the shared inputs (W(q), q-maps, pair elements of the widest band
window) are uploaded once and sliced per problem on the device."""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L
from .bse import (PRECISIONS, TYPES, _dev, coulomb_v0, device_vbar_probe,
                  kernel_prefactor)


class Batch:
    def __init__(self, members: list, precision: str = "fp64", nbranch: int = 16,
                 bse_type: str = "singlet", device: str = "cuda"):
        from . import tune
        tune.load()  # the autotuner's tile choices, when a table is present
        dv = self.device = torch.device(device)
        c128, f64 = torch.complex128, torch.float64
        self.members = members
        master = members[0].get("master", members[0])
        self.shared = {"W": _dev(master["W"], c128, dv),
                       "qmap": _dev(master["qmap"], torch.int32, dv),
                       "qramap": _dev(master["qramap"], torch.int32, dv)}
        for k in ("Mvv", "Mcc", "Ncv", "Nvc"):
            if k in master and master[k] is not None:
                self.shared[k] = _dev(master[k], c128, dv)
        self.t, self.descs, self.inputs = [], [], []
        self.pref, self.eta, self.nw = [], [], []
        for d in members:
            w = d["workload"]
            nv, nc = w.nv, w.nc
            t = {"eps_v": _dev(d["eps_v"], f64, dv), "eps_c": _dev(d["eps_c"], f64, dv),
                 "Mcv": _dev(d["Mcv"], c128, dv),
                 "Mvv": self.shared["Mvv"][:, :nv, :nv, :].contiguous(),
                 "Mcc": self.shared["Mcc"][:, :nc, :nc, :].contiguous()}
            full = w.coupling == "full"
            if full:
                t["Ncv"] = self.shared["Ncv"][:, :nc, :nv, :].contiguous()
                t["Nvc"] = self.shared["Nvc"][:, :nv, :nc, :].contiguous()
            t["vbar"], t["probe"] = device_vbar_probe(d["gvec"], d["alat"], w.q, w.n, w.ng,
                                                      t["Mcv"], dv)
            t["omega"] = _dev(d["omega"], f64, dv)
            n = w.n
            t["H0"] = torch.empty((n, n), dtype=c128, device=dv)
            t["H1"] = torch.empty((n, n), dtype=c128, device=dv) if full else None
            t["E"] = torch.empty(n, dtype=f64, device=dv)
            t["osc"] = torch.empty(n, dtype=f64, device=dv)
            t["eps"] = torch.empty(w.nw, dtype=c128, device=dv)
            kap = kernel_prefactor(w.kernel_scale, w.nk, d["cell_volume"])
            self.pref.append(2.0 * kap * coulomb_v0(w.q))
            self.eta.append(w.eta)
            self.nw.append(w.nw)
            prec, terms = PRECISIONS[precision]
            self.descs.append(L.BseDesc(nk=w.nk, nv=nv, nc=nc, ng=w.ng,
                                        coupling=L.BSE_FULL if full else L.BSE_TDA,
                                        type=TYPES[bse_type], prec=prec, split_terms=terms,
                                        kappa=kap, scissor=w.scissor, ld=n))
            p = lambda k: t[k].data_ptr() if t.get(k) is not None else None  # noqa: E731
            self.inputs.append(L.BseInputs(
                eps_v=p("eps_v"), eps_c=p("eps_c"), Mcv=p("Mcv"), Mvv=p("Mvv"), Mcc=p("Mcc"),
                Ncv=p("Ncv"), Nvc=p("Nvc"), W=self.shared["W"].data_ptr(), vbar=p("vbar"),
                qmap=self.shared["qmap"].data_ptr(),
                qramap=self.shared["qramap"].data_ptr() if full else None,
                nq=int(master["W"].shape[0]), reserved=0))
            self.t.append(t)
        self.nbranch = nbranch
        self.ws = torch.empty(max(1, L.bse_batch_workspace_size(self.descs, nbranch)),
                              dtype=torch.uint8, device=dv)
        self.info = torch.zeros(len(members), dtype=torch.int32, device=dv)
        self.handle = L.bse_batch_create(self.descs, nbranch)
        self.captured = False
        # capture and replay on a stream of our own (default priority): the
        # legacy NULL stream cannot be captured
        self.cs = torch.cuda.Stream(device=dv)

    def _ptr(self, key):
        return [t[key].data_ptr() if t[key] is not None else None for t in self.t]

    @staticmethod
    def stream() -> int:
        return torch.cuda.current_stream().cuda_stream

    def capture(self) -> None:
        self.cs.wait_stream(torch.cuda.current_stream())
        L.bse_batch_capture(self.handle, self.inputs, self._ptr("H0"), self._ptr("H1"),
                            self._ptr("E"), self._ptr("probe"), self._ptr("osc"), self.pref,
                            self.eta, self.nw, self._ptr("omega"), self._ptr("eps"),
                            self.ws.data_ptr(), self.ws.numel(), self.info.data_ptr(),
                            self.cs.cuda_stream)
        self.captured = True

    def run(self) -> None:
        """One replay of the graph (captured on first use), ordered after the
        work already on the current stream; the current stream waits for it."""
        if not self.captured:
            self.capture()
        cur = torch.cuda.current_stream()
        self.cs.wait_stream(cur)
        L.bse_batch_run(self.handle, self.cs.cuda_stream)
        cur.wait_stream(self.cs)

    def run_sequential(self) -> None:
        """The same problems one after another through the plain entry points."""
        s = self.stream()
        ws_bytes = self.ws.numel() // max(1, min(self.nbranch, len(self.t)))
        for i, t in enumerate(self.t):
            d, n = self.descs[i], int(self.descs[i].nk * self.descs[i].nv * self.descs[i].nc)
            info = self.info.data_ptr() + 4 * i
            L.bse_build(d, self.inputs[i], t["H0"].data_ptr(),
                        t["H1"].data_ptr() if t["H1"] is not None else 0,
                        self.ws.data_ptr(), ws_bytes, info, s)
            L.bse_solve(d, t["H0"].data_ptr(), t["H1"].data_ptr() if t["H1"] is not None else 0,
                        t["E"].data_ptr(), 0, 0, n, t["probe"].data_ptr(), t["osc"].data_ptr(),
                        self.ws.data_ptr(), ws_bytes, info, s)
            L.bse_spectrum(n, t["E"].data_ptr(), t["osc"].data_ptr(), self.pref[i], self.eta[i],
                           self.nw[i], t["omega"].data_ptr(), t["eps"].data_ptr(), s)

    def set_precision(self, precision: str) -> None:
        """Switch the assembly arithmetic (needs a new capture)."""
        prec, terms = PRECISIONS[precision]
        for d in self.descs:
            d.prec, d.split_terms = prec, terms
        L.bse_batch_destroy(self.handle)
        self.handle = L.bse_batch_create(self.descs, self.nbranch)
        self.captured = False

    def results(self) -> list:
        torch.cuda.synchronize()
        info = self.info.cpu().numpy()
        if np.any(info != 0):
            raise L.BseError(f"device status info = {info.tolist()}")
        return [{"E": t["E"].cpu().numpy(), "osc": t["osc"].cpu().numpy(),
                 "eps": t["eps"].cpu().numpy()} for t in self.t]

    def close(self) -> None:
        if self.handle:
            L.bse_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def main() -> int:
    """Replay one batch workload's graph (one branch per problem, the stored
    tuning table) and print the time per replay:

        python -m paper_1904_05575_amd.batch [--workload batch16_k6_g89] [--replays 3]
                                             [--precision fp64]
    """
    import argparse
    import json
    import sys
    import time

    from bse_synth import BATCHES, make_batch_inputs
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="batch16_k6_g89", choices=sorted(BATCHES))
    ap.add_argument("--replays", type=int, default=3)
    ap.add_argument("--precision", default="fp64", choices=sorted(PRECISIONS))
    args = ap.parse_args()
    ms = make_batch_inputs(BATCHES[args.workload])
    B = Batch(ms, precision=args.precision, nbranch=len(ms))
    B.run()  # capture and a first replay
    B.results()
    times = []
    for _ in range(args.replays):
        t0 = time.perf_counter()
        B.run()
        torch.cuda.synchronize()
        times.append(1e3 * (time.perf_counter() - t0))
        print(f"[batch] replay {len(times)}: {times[-1]:.1f} ms", file=sys.stderr, flush=True)
    B.results()  # raises on a device error
    B.close()
    print(json.dumps({"workload": args.workload, "problems": len(ms),
                      "precision": args.precision, "replay_ms": [round(t, 1) for t in times]}))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())

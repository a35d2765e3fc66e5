"""Seeded synthetic inputs of the BSE hot path.

Draws the quantities the paper's earlier tasks would produce (Kohn-Sham
energies, plane-wave pair matrix elements, the static screened interaction)
as random arrays of the right shapes and magnitudes.  No step of the BSE
method itself happens here.

Recipe (all complex draws are standard complex normal, E|z|^2 = 1):
  eps_v[k, v] ~ U(eps_v_range)          (or a flat core level)
  eps_c[k, c] ~ U(eps_c_range)
  Mcv[a, G]        ~ CN / (1 + |G+Q|^2)  (or exp(-|G+Q|^2 / (2 w^2)) for core)
  Mvv[p, v, v', G] ~ CN / (1 + |G|^2)    (pairs p = (ik <= ik'))
  Mcc[p, c, c', G] ~ CN / (1 + |G|^2)
                   (or, for mcc_generated workloads, only its description: the
                   envelope 1 / (1 + |G|^2) and a 64-bit key; the values are
                   drawn where they are used by a counter-based generator,
                   Philox4x32-10 at counter (p, c, c', G) + Box-Muller, which
                   each consumer implements from its published definition)
  Ncv[p, c, v', G], Nvc[p, v, c', G]  as Mvv (full BSE only)
  Dcv[a, j] ~ CN / (eps_c - eps_v)      (dipole elements along x, y, z: a
                                         momentum element over the transition's
                                         energy difference, the optical limit)
  W[q] = v^1/2(q+G) (I + L_q L_q^H)^-1 v^1/2(q+G'),  L_q ~ 0.3 CN (NG x 8),
         v(p) = 4 pi / |p|^2 with |p|^2 replaced by 0.01 at p = 0.
Workloads with orbitals > 0 carry, instead of the pair elements and M_cv,
synthetic orbitals: plane-wave coefficients C[k, n, K] on the sphere of the
first `orbitals` reciprocal vectors K (occupied bands first), complex normal
times 1/(1 + |K|^2), each orbital normalised (sum_K |C|^2 = 1) but the bands
of one k not orthogonalised (so that the G = 0 element between an occupied
and an unoccupied band at the same k, the Q = 0 probe, does not vanish);
`kvec` holds the sphere's integer coordinates, `gvec` those of the G-set.
Inputs of the RPA screening (make_screening_inputs): the workload's energies
and, for every q of the mesh and k, pair elements between the bands at k and
at k + q,
  Svc[q, k, v, c, G], Scv[q, k, c, v, G] ~ CN |p| / (1 + |p|^2),  p = q + G
         (|p| replaced by 0.1 at p = 0; the factor |p| mimics M ~ q.D near
         p = 0, which keeps v |M|^2 finite).
Transition index a = (ik * nv + iv) * nc + ic.

Large arrays are drawn in fixed-size chunks, each from its own Philox stream
keyed by (seed, array, chunk), so the result does not depend on the number of
threads.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import lattice
from .workloads import Workload

_KIND = {"eps_v": 1, "eps_c": 2, "Mcv": 3, "Mvv": 4, "Mcc": 5, "Ncv": 6, "Nvc": 7, "L": 8,
         "Dcv": 9, "Svc": 10, "Scv": 11, "C": 12}
_CHUNK_ROWS = 1024
_INV_SQRT2 = 1.0 / np.sqrt(2.0)


def _rng(seed: int, kind: str, chunk: int) -> np.random.Generator:
    ss = np.random.SeedSequence(entropy=seed, spawn_key=(_KIND[kind], chunk))
    return np.random.Generator(np.random.Philox(ss))


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _complex_rows(seed: int, kind: str, shape: tuple, envelope: np.ndarray) -> np.ndarray:
    """Complex normal array of `shape` (rows first), times a real envelope that
    broadcasts against one row."""
    out = np.empty(shape, dtype=np.complex128)
    rows = shape[0]
    nchunks = (rows + _CHUNK_ROWS - 1) // _CHUNK_ROWS
    env = (envelope * _INV_SQRT2).astype(np.float64)

    def fill(ci: int) -> None:
        lo, hi = ci * _CHUNK_ROWS, min(rows, (ci + 1) * _CHUNK_ROWS)
        blk = out[lo:hi]
        _rng(seed, kind, ci).standard_normal(out=blk.view(np.float64))
        blk *= env

    if nchunks == 1:
        fill(0)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(fill, range(nchunks)))
    return out


def screened_interaction(w: Workload) -> np.ndarray:
    """W[iq, G, G'] for every q class of lattice.q_maps (the BSE's input from
    screening): the q-mesh and, for a generic k-shift, the second set."""
    ng, n = w.ng, w.mesh
    G = lattice.gcart(ng)
    qc = lattice.qset_cart(n, w.kshift)
    nq = len(qc)
    L = _complex_rows(w.seed, "L", (nq, ng, 8), np.full((ng, 8), 0.3))
    W = np.empty((nq, ng, ng), dtype=np.complex128)
    eye = np.eye(ng)
    for iq in range(nq):
        p2 = np.sum((qc[iq][None, :] + G) ** 2, axis=1)
        p2 = np.where(p2 < 1e-12, 0.01, p2)
        sv = np.sqrt(4.0 * np.pi / p2)
        Lq = L[iq]
        inv = np.linalg.inv(eye + Lq @ Lq.conj().T)
        inv = 0.5 * (inv + inv.conj().T)
        W[iq] = sv[:, None] * inv * sv[None, :]
    return W


def mcc_key(w: Workload) -> int:
    """64-bit key of the drawn Mcc: low word the workload seed, high word the
    array kind."""
    return (w.seed & 0xFFFFFFFF) | (_KIND["Mcc"] << 32)


def make_inputs(w: Workload, want_pairs: bool = True) -> dict:
    """All inputs of one BSE problem as NumPy arrays (host memory)."""
    nk, nv, nc, ng = w.nk, w.nv, w.nc, w.ng
    G = lattice.gcart(ng)
    Q = np.asarray(w.q, dtype=np.float64)
    out: dict = {"workload": w}
    g1 = _rng(w.seed, "eps_v", 0)
    if w.core_level is not None:
        out["eps_v"] = np.full((nk, nv), float(w.core_level))
    else:
        out["eps_v"] = g1.uniform(w.eps_v_range[0], w.eps_v_range[1], size=(nk, nv))
    out["eps_c"] = _rng(w.seed, "eps_c", 0).uniform(w.eps_c_range[0], w.eps_c_range[1],
                                                    size=(nk, nc))
    gq2 = np.sum((G + Q[None, :]) ** 2, axis=1)
    if w.mcv_gauss_width is not None:
        env_cv = np.exp(-gq2 / (2.0 * w.mcv_gauss_width ** 2))
    else:
        env_cv = 1.0 / (1.0 + gq2)
    out["Mcv"] = _complex_rows(w.seed, "Mcv", (w.n, ng), env_cv)
    de = (out["eps_c"][:, None, :] - out["eps_v"][:, :, None]).reshape(w.n)
    out["Dcv"] = _complex_rows(w.seed, "Dcv", (w.n, 3), np.ones(3)) / de[:, None]
    env = 1.0 / (1.0 + np.sum(G ** 2, axis=1))
    if w.orbitals:
        # orbitals instead of pair elements (the consumers form M, N, M_cv)
        Kc = lattice.gcart(w.orbitals)
        nb = nv + nc
        C = _complex_rows(w.seed, "C", (nk * nb, w.orbitals),
                          1.0 / (1.0 + np.sum(Kc ** 2, axis=1)))
        C /= np.linalg.norm(C, axis=1, keepdims=True)
        out["C"] = C.reshape(nk, nb, w.orbitals)
        out["kvec"] = lattice.gvectors(w.orbitals)
        del out["Mcv"]
        want_pairs = False
    if want_pairs:
        P = w.npairs
        out["Mvv"] = _complex_rows(w.seed, "Mvv", (P, nv, nv, ng), env)
        if w.mcc_generated:
            out["Mcc"] = None
            out["mcc_env"] = env.astype(np.float64)
            out["mcc_key"] = mcc_key(w)
        else:
            out["Mcc"] = _complex_rows(w.seed, "Mcc", (P, nc, nc, ng), env)
        if w.coupling == "full":
            out["Ncv"] = _complex_rows(w.seed, "Ncv", (P, nc, nv, ng), env)
            out["Nvc"] = _complex_rows(w.seed, "Nvc", (P, nv, nc, ng), env)
    out["W"] = screened_interaction(w) if (want_pairs or w.orbitals) else None
    qmap, qramap = lattice.q_maps(w.mesh, w.kshift)
    out["qmap"], out["qramap"] = qmap, qramap
    out["gvec"] = lattice.gvectors(ng)
    out["kcoords"] = lattice.kmesh(w.mesh)
    out["omega"] = np.linspace(w.wmin, w.wmax, w.nw)
    out["alat"] = lattice.A_LATT
    out["cell_volume"] = lattice.cell_volume()
    return out


def make_batch_inputs(bw) -> list:
    """Inputs of every member of a BatchWorkload.  W(q), the q-maps and the
    pair arrays come from the master (widest band window); member m takes the
    first nv occupied and nc unoccupied bands of them (NumPy views)."""
    master = make_inputs(bw.master)
    out = []
    for w in bw.members:
        d = make_inputs(w, want_pairs=False)
        d["W"] = master["W"]
        d["qmap"], d["qramap"] = master["qmap"], master["qramap"]
        nv, nc = w.nv, w.nc
        d["Mvv"] = master["Mvv"][:, :nv, :nv, :]
        d["Mcc"] = master["Mcc"][:, :nc, :nc, :]
        if w.coupling == "full":
            d["Ncv"] = master["Ncv"][:, :nc, :nv, :]
            d["Nvc"] = master["Nvc"][:, :nv, :nc, :]
        d["master"] = master
        out.append(d)
    return out


def make_screening_inputs(w: Workload) -> dict:
    """Inputs of the RPA screening on the workload's mesh and bands: energies,
    the index of k + q on the mesh, and the pair elements of both orders."""
    base = make_inputs(w, want_pairs=False)
    n, nk, nv, nc, ng = w.mesh, w.nk, w.nv, w.nc, w.ng
    km = lattice.kmesh(n)
    kq = lattice.mesh_index(km[None, :, :] + km[:, None, :], n).astype(np.int32)  # [q, k]
    qc = lattice.centred_cart(km, n)
    G = lattice.gcart(ng)
    p = np.sqrt(np.sum((qc[:, None, :] + G[None, :, :]) ** 2, axis=2))       # [q, G]
    p = np.where(p < 1e-6, 0.1, p)
    env = p / (1.0 + p ** 2)
    out = {"workload": w, "eps_v": base["eps_v"], "eps_c": base["eps_c"], "kqmap": kq,
           "qcart": qc, "gvec": base["gvec"], "alat": base["alat"],
           "cell_volume": base["cell_volume"]}
    for kind, b1, b2 in (("Svc", nv, nc), ("Scv", nc, nv)):
        a = np.empty((nk, nk, b1, b2, ng), dtype=np.complex128)

        def fill(iq: int) -> None:  # one Philox stream per q
            blk = a[iq].reshape(-1).view(np.float64)
            _rng(w.seed * 4096 + iq, kind, 0).standard_normal(out=blk)
            a[iq] *= env[iq] * _INV_SQRT2

        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(fill, range(nk)))
        out[kind] = a
    return out

"""Plane-wave pair elements from orbital coefficients (test infrastructure).

Only the tests and the benchmark's CPU baseline use this module; the GPU
library never calls it.

The paper (Sec. 4.1) forms the BSE's plane-wave matrix elements from the
orbitals: M_mn,k(G, q) = <m k| exp(-i(G+q) r) |n k+q>, and the modified
elements N_mn,k(G, q) = <m k| exp(-i(G+q) r) |(n k+q)*>, each a sum over the
orbitals' basis coefficients.  For orbitals expanded in plane waves only,
    phi_n,k(r) = Omega^-1/2 sum_K C_n,k(K) exp(i (k + K) r),
the integral over the cell keeps the terms whose wave vectors cancel, which
leaves the restricted sums written out here:
    M_mn(k, k', G) = sum_K conj(C_m,k(K)) C_n,k'(K + G)      (q = k' - k)
    N_mn(k, k', G) = sum_K conj(C_m,k(K)) conj(C_n,k'(-K - G))  (q = -k - k')
with K over the orbitals' plane-wave sphere and a term dropped when K + G
(or -K - G) lies outside it.  The BSE inputs follow for every pair
p = (ik <= ik'), v occupied and c unoccupied bands (occupied first in C):
    Mvv[p][v][v'][G] = M_vv'(k, k', G)      Mcc[p][c][c'][G] = M_cc'(k, k', G)
    Ncv[p][c][v'][G] = N_cv'(k, k', G)      Nvc[p][v][c'][G] = N_vc'(k, k', G)
    Mcv[(k, v, c)][G] = M_vc(k, k, G)       (momentum transfer Q = 0)
The partner of each K is looked up by the integer coordinates of the
sphere's vectors; for each G the sum over K is one product of the two bands'
coefficient rows.
"""
from __future__ import annotations

import numpy as np


def _lookup(kvec: np.ndarray) -> dict:
    """Position of every integer vector of the orbital sphere."""
    return {tuple(int(x) for x in v): i for i, v in enumerate(kvec)}


def partner(kvec: np.ndarray, gvec: np.ndarray, modified: bool) -> np.ndarray:
    """[NG][NK]: position in the sphere of K + G (modified: of -K - G), or -1
    when it lies outside."""
    pos = _lookup(kvec)
    out = -np.ones((len(gvec), len(kvec)), dtype=np.int64)
    for g, G in enumerate(gvec):
        for a, K in enumerate(kvec):
            tgt = tuple(int(x) for x in ((-K - G) if modified else (K + G)))
            out[g, a] = pos.get(tgt, -1)
    return out


def pair_element(Ck: np.ndarray, Ckp: np.ndarray, kvec: np.ndarray, gvec: np.ndarray,
                 modified: bool, table: np.ndarray | None = None) -> np.ndarray:
    """M (modified=False) or N (modified=True) for all band pairs of one
    k-pair: out[m][n][G] for Ck [nbm][NK] (bands at k) and Ckp [nbn][NK]
    (bands at k').  kvec [NK][3], gvec [NG][3]: integer coordinates of the
    sphere and of the G-set in one lattice basis.  For each G the sum runs
    over the K whose partner is in the sphere."""
    tab = partner(kvec, gvec, modified) if table is None else table
    nbm, nbn, ng = Ck.shape[0], Ckp.shape[0], len(gvec)
    out = np.zeros((nbm, nbn, ng), dtype=np.complex128)
    for g in range(ng):
        a = np.nonzero(tab[g] >= 0)[0]
        b = tab[g, a]
        right = np.conj(Ckp[:, b]) if modified else Ckp[:, b]
        out[:, :, g] = np.conj(Ck[:, a]) @ right.T
    return out


def pair_elements_batch(Ca: np.ndarray, Cb: np.ndarray, table: np.ndarray,
                        modified: bool) -> np.ndarray:
    """pair_element for a batch of k-pairs at once: Ca [P][nbm][NK] (bands at
    k), Cb [P][nbn][NK] (bands at k') -> [P][nbm][nbn][NG], the same sum per G."""
    P, nbm, _ = Ca.shape
    nbn, ng = Cb.shape[1], table.shape[0]
    out = np.zeros((P, nbm, nbn, ng), dtype=np.complex128)
    for g in range(ng):
        a = np.nonzero(table[g] >= 0)[0]
        b = table[g, a]
        right = np.conj(Cb[:, :, b]) if modified else Cb[:, :, b]
        out[:, :, :, g] = np.conj(Ca[:, :, a]) @ np.swapaxes(right, 1, 2)
    return out


def bse_pair_arrays(C: np.ndarray, nv: int, kvec: np.ndarray, gvec: np.ndarray,
                    coupling: bool = True, pairs: np.ndarray | None = None,
                    chunk: int = 4096) -> dict:
    """Mcv, Mvv, Mcc (and Ncv, Nvc) of the BSE from orbital coefficients
    C [nk][nv + nc][NK] (occupied bands first); pairs (ik, ik') with ik <= ik'
    in row-major order, or the given subset."""
    nk, nb, _ = C.shape
    nc = nb - nv
    ng = len(gvec)
    if pairs is None:
        ik, jk = np.triu_indices(nk)
        pairs = np.stack([ik, jk], axis=1)
    P = len(pairs)
    tp = partner(kvec, gvec, modified=False)
    tm = partner(kvec, gvec, modified=True)
    out = {"Mvv": np.empty((P, nv, nv, ng), dtype=np.complex128),
           "Mcc": np.empty((P, nc, nc, ng), dtype=np.complex128)}
    if coupling:
        out["Ncv"] = np.empty((P, nc, nv, ng), dtype=np.complex128)
        out["Nvc"] = np.empty((P, nv, nc, ng), dtype=np.complex128)
    for p0 in range(0, P, chunk):
        sl = slice(p0, min(P, p0 + chunk))
        Ca, Cb = C[pairs[sl, 0]], C[pairs[sl, 1]]
        Mab = pair_elements_batch(Ca, Cb, tp, modified=False)
        out["Mvv"][sl] = Mab[:, :nv, :nv]
        out["Mcc"][sl] = Mab[:, nv:, nv:]
        if coupling:
            Nab = pair_elements_batch(Ca, Cb, tm, modified=True)
            out["Ncv"][sl] = Nab[:, nv:, :nv]
            out["Nvc"][sl] = Nab[:, :nv, nv:]
    Mcv = pair_elements_batch(C, C, tp, modified=False)[:, :nv, nv:]
    out["Mcv"] = Mcv.reshape(nk * nv * nc, ng)
    return out


def complete_inputs(d: dict) -> dict:
    """The inputs of an orbital workload with the pair elements the oracle
    forms from its orbitals added (a new dict; the arrays of d are shared)."""
    w = d["workload"]
    out = dict(d)
    out.update(bse_pair_arrays(d["C"], w.nv, d["kvec"], d["gvec"], coupling=w.coupling == "full"))
    if w.coupling != "full":
        out["Ncv"] = out["Nvc"] = None
    return out

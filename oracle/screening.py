"""Plain FP64 CPU oracle of the static RPA screening (test infrastructure:
only the tests, the smoke check and the benchmark's CPU-baseline leg use it;
the GPU library never calls it).

Follows Sec. 4.2 of the paper (Vorwerk et al., "Bethe-Salpeter equation for
absorption and scattering spectroscopy: implementation in the exciting
code"): the RPA dielectric matrix
    eps_GG'(q, w) = delta_GG' - (1/V_c) v_G'(q) sum_{ijk}
                    (f_j,k+q - f_i,k) / (e_j,k+q - e_i,k - w) conj(M^G_ij) M^G'_ij
and the screened interaction w_GG'(q) = v_G(q) eps^-1_GG'(q, w = 0)
(eq. wggq), which the direct terms of the BSE kernel contract (eqs. wrrm,
wrabar).

Readings (listed with their reasons in the design notes): an insulator at
zero temperature, f = 1 in the occupied and 0 in the unoccupied bands, so
only the pairs (occupied at k, unoccupied at k + q) and (unoccupied at k,
occupied at k + q) contribute; no spin factor beyond the printed formula;
energies in eV converted to Hartree (1/V_c in bohr^-3, v(p) = 4 pi / |p|^2
in bohr^-2 with |p|^2 replaced by 0.01 at p = 0, as for the BSE inputs).

Pinned in tests/test_oracle_screening.py against a literal loop over every
band pair with its occupation factors, the Sherman-Morrison closed form of a
single transition, the bare limit and the ordering 0 < W <= v.
"""
from __future__ import annotations

import numpy as np

HARTREE_EV = 27.211386245988


def coulomb(qcart: np.ndarray, gcart: np.ndarray) -> np.ndarray:
    """v[q, G] = 4 pi / |q + G|^2, |q + G|^2 -> 0.01 at q + G = 0."""
    p2 = np.sum((qcart[:, None, :] + gcart[None, :, :]) ** 2, axis=2)
    return 4.0 * np.pi / np.where(p2 < 1e-12, 0.01, p2)


def chi_sum(Svc, Scv, eps_v, eps_c, kqmap, iq: int, inv_vc: float) -> np.ndarray:
    """X[G, G'] = (1/V_c) sum_ijk F_ij conj(M^G_ij) M^G'_ij at w = 0 for one q,
    F_ij = (f_j,k+q - f_i,k) / (e_j,k+q - e_i,k) in 1/Hartree."""
    ng = Svc.shape[-1]
    X = np.zeros((ng, ng), dtype=np.complex128)
    for k in range(Svc.shape[1]):
        kq = kqmap[iq, k]
        # i occupied at k, j unoccupied at k+q: f_j - f_i = -1
        F = -1.0 / ((eps_c[kq][None, :] - eps_v[k][:, None]) / HARTREE_EV)       # [v, c]
        M = Svc[iq, k].reshape(-1, ng)
        X += (M.conj().T * F.reshape(-1)) @ M
        # i unoccupied at k, j occupied at k+q: f_j - f_i = +1
        F = 1.0 / ((eps_v[kq][None, :] - eps_c[k][:, None]) / HARTREE_EV)        # [c, v]
        M = Scv[iq, k].reshape(-1, ng)
        X += (M.conj().T * F.reshape(-1)) @ M
    return inv_vc * X


def dielectric_matrix(X: np.ndarray, v: np.ndarray) -> np.ndarray:
    """eps[G, G'] = delta_GG' - v_G' X[G, G']."""
    return np.eye(len(v)) - X * v[None, :]


def screened_w(eps: np.ndarray, v: np.ndarray) -> np.ndarray:
    """w[G, G'] = v_G eps^-1[G, G']  (eq. wggq)."""
    return v[:, None] * np.linalg.inv(eps)


def screening(inputs: dict) -> np.ndarray:
    """W[q, G, G'] for every q of the mesh."""
    from bse_synth import lattice
    w = inputs["workload"]
    inv_vc = 1.0 / (w.nk * inputs["cell_volume"])
    v = coulomb(inputs["qcart"], lattice.gcart(w.ng))
    out = np.empty((w.nk, w.ng, w.ng), dtype=np.complex128)
    for iq in range(w.nk):
        X = chi_sum(inputs["Svc"], inputs["Scv"], inputs["eps_v"], inputs["eps_c"],
                    inputs["kqmap"], iq, inv_vc)
        out[iq] = screened_w(dielectric_matrix(X, v[iq]), v[iq])
    return out

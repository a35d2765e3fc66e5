"""Plain FP64 CPU oracle of the optical-limit and scattering observables
(test infrastructure: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the GPU library never calls it).

Follows Sec. 4.4 of the paper (Vorwerk et al., "Bethe-Salpeter equation for
absorption and scattering spectroscopy: implementation in the exciting
code"):

* transition coefficients per Cartesian direction i (eq. tlambdai):
      t_li = -i sum_a conj((X+Y)_al) conj(D_ai)
  with D the dipole elements of eq. dipolfromp;
* the macroscopic dielectric tensor (eq. epsmij):
      eps^ij(w) = delta_ij - pref sum_l conj(t_li) t_lj
                  [1/(w - E_l + i eta) - 1/(w + E_l + i eta)]
  (the second denominator of the printed equation, garbled with a doubled i,
  is read as -w - E_l - i eta, the form of eq. epsmtensor; pref = 2 kappa 4 pi
  with spin factor 2 and 1/V_c as in the scalar spectrum);
* the electron energy-loss function L = -Im 1/eps_M (eq. Lofeps) and the
  dynamic structure factor S(Q, w) = -(1/pi) v_G(q)^-1 Im 1/eps_M.

Pinned in tests/test_oracle_observables.py against the resolvent definition
of eps_M (contraction of the tensor with complex direction vectors), the
closed form of a single pole's loss function, the f-sum rule of S, and the
identity X+Y = 1.
"""
from __future__ import annotations

import numpy as np


def transition_coefficients(XpY: np.ndarray, D: np.ndarray) -> np.ndarray:
    """t[l, i] = -i sum_a conj(XpY[a, l]) conj(D[a, i])  (eq. tlambdai)."""
    return -1j * (XpY.conj().T @ D.conj())


def dielectric_tensor(E: np.ndarray, t: np.ndarray, omega: np.ndarray, eta: float,
                      pref: float) -> np.ndarray:
    """eps[w, i, j] of eq. epsmij from energies E[l] and coefficients t[l, i]."""
    z = omega[:, None] + 1j * eta
    g = 1.0 / (z - E[None, :]) - 1.0 / (z + E[None, :])          # [w, l]
    h = t.conj()[:, :, None] * t[:, None, :]                       # [l, i, j]
    nd = t.shape[1]
    return np.eye(nd)[None, :, :] - pref * np.einsum("wl,lij->wij", g, h)


def contract(eps: np.ndarray, u: np.ndarray) -> np.ndarray:
    """sum_ij conj(u_i) eps^ij u_j for every frequency (q-hat^T eps q-hat for
    a real direction q-hat, the first line of eq. epsmtensor)."""
    return np.einsum("i,wij,j->w", u.conj(), eps, u)


def loss_function(eps: np.ndarray) -> np.ndarray:
    """L = -Im 1/eps_M  (eq. Lofeps)."""
    return -np.imag(1.0 / eps)


def dynamic_structure_factor(eps: np.ndarray, v: float) -> np.ndarray:
    """S(Q, w) = -(1/pi) v_G(q)^-1 Im 1/eps_M(q, w), v = v_G(q)."""
    return -np.imag(1.0 / eps) / (np.pi * v)


def tensor_prefactor(inputs: dict) -> float:
    """2 kappa 4 pi: spin factor 2, 1/V_c and the 4 pi that is left of v(q)
    once M = i q.D cancels its 1/q^2 (eq. mofd)."""
    from .bse_oracle import kappa
    return 2.0 * kappa(inputs) * 4.0 * np.pi

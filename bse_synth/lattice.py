"""Geometry of the synthetic crystal: fcc lattice, its reciprocal G-shells and a
Gamma-centred k-mesh.

This module only lays out the index spaces the BSE inputs live on (plane-wave
set, k-points, momentum-transfer classes).  It holds none of the method's
arithmetic and is shared by the input generator and the host code of both
sides.

Units: bohr for lengths, bohr^-1 for wave vectors.
"""
from __future__ import annotations

import numpy as np

# Lattice constant of the synthetic fcc crystal (bohr); close to silicon, the
# paper's loss-function example (Sec. 5.4).
A_LATT = 10.263

# |G|^2 / (2 pi / a)^2 bounds that close a shell of the bcc reciprocal lattice,
# with the number of G-vectors inside (plane-wave cut-off gqmax, Appendix B).
SHELL_BOUND = {1: 0, 9: 3, 15: 4, 27: 8, 51: 11, 59: 12, 65: 16, 89: 19, 113: 20,
               137: 24, 169: 27}


def cell_volume(a: float = A_LATT) -> float:
    """Primitive fcc cell volume a^3/4 (bohr^3)."""
    return a ** 3 / 4.0


def recip_basis(a: float = A_LATT) -> np.ndarray:
    """Rows b1, b2, b3 of the fcc reciprocal basis (bohr^-1)."""
    s = 2.0 * np.pi / a
    return s * np.array([[-1.0, 1.0, 1.0], [1.0, -1.0, 1.0], [1.0, 1.0, -1.0]])


def gvectors(ng: int) -> np.ndarray:
    """Integer (h, k, l) of the ng shortest G = (2 pi / a)(h, k, l) of the bcc
    reciprocal lattice (h, k, l all even or all odd), ordered by
    (|G|^2, h, k, l).  ng must close a shell."""
    if ng not in SHELL_BOUND:
        raise ValueError(f"ng={ng} does not close a G-shell; allowed {sorted(SHELL_BOUND)}")
    bound = SHELL_BOUND[ng]
    r = int(np.ceil(np.sqrt(bound))) + 1
    out = []
    for h in range(-r, r + 1):
        for k in range(-r, r + 1):
            for l in range(-r, r + 1):
                if (h % 2 == k % 2 == l % 2) and h * h + k * k + l * l <= bound:
                    out.append((h * h + k * k + l * l, h, k, l))
    out.sort()
    g = np.array([o[1:] for o in out], dtype=np.int64)
    assert len(g) == ng, (len(g), ng)
    return g


def gcart(ng: int, a: float = A_LATT) -> np.ndarray:
    """Cartesian G-vectors (ng, 3) in bohr^-1."""
    return gvectors(ng).astype(np.float64) * (2.0 * np.pi / a)


def kmesh(n: int) -> np.ndarray:
    """Integer mesh coordinates (n^3, 3) of a Gamma-centred n x n x n mesh;
    k-point ik = (i1 * n + i2) * n + i3 sits at sum_j (i_j / n) b_j."""
    i = np.arange(n)
    g = np.stack(np.meshgrid(i, i, i, indexing="ij"), axis=-1).reshape(-1, 3)
    return g.astype(np.int64)


def mesh_index(coords: np.ndarray, n: int) -> np.ndarray:
    """Flat mesh index of integer mesh coordinates (taken modulo n)."""
    c = np.mod(coords, n)
    return (c[..., 0] * n + c[..., 1]) * n + c[..., 2]


def centred_cart(coords: np.ndarray, n: int, a: float = A_LATT) -> np.ndarray:
    """Cartesian vector of mesh coordinates, each residue mapped to the centred
    range [-n/2, n/2) before the sum over the reciprocal basis."""
    c = np.mod(coords, n)
    c = np.mod(c + n // 2, n) - n // 2
    return (c.astype(np.float64) / n) @ recip_basis(a)


def pair_count(nk: int) -> int:
    """Number of k-pairs (ik <= ik')."""
    return nk * (nk + 1) // 2


def pair_list(nk: int) -> np.ndarray:
    """(P, 2) array of the pairs (ik, ik') with ik <= ik' in row-major order;
    row p is pair p of every pair-indexed input array."""
    ik, jk = np.triu_indices(nk)
    return np.stack([ik, jk], axis=1).astype(np.int64)


def _second_set(shift) -> tuple[bool, np.ndarray]:
    """For k = (i + s)/n: -k-k' = (-(i + i') - 2s)/n.  Returns whether 2s is
    integral (then -k-k' is on the q-mesh itself) and 2s rounded."""
    m = 2.0 * np.asarray(shift, dtype=np.float64)
    return not np.allclose(m, np.round(m), atol=1e-12), np.round(m).astype(np.int64)


def q_maps(n: int, shift=(0.0, 0.0, 0.0)) -> tuple[np.ndarray, np.ndarray]:
    """Momentum-transfer classes of k-pairs on the mesh:
    qmap[ik, ik'] = index of k - k' (always on the q-mesh {j/n}) and
    qramap[ik, ik'] = index of -k - k': on the q-mesh when 2 shift is integral,
    else on the second set {(j - 2 shift)/n}, whose entries follow the Nk
    entries of the first in W (index Nk + j)."""
    km = kmesh(n)
    qmap = mesh_index(km[:, None, :] - km[None, :, :], n)
    second, m = _second_set(shift)
    if second:
        qramap = n ** 3 + mesh_index(-km[:, None, :] - km[None, :, :], n)
    else:
        qramap = mesh_index(-km[:, None, :] - km[None, :, :] - m, n)
    return qmap.astype(np.int32), qramap.astype(np.int32)


def qset_cart(n: int, shift=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Cartesian q-vectors (centred) of every class of q_maps: the q-mesh, then
    (for a generic shift) the second set (j - 2 shift)/n."""
    km = kmesh(n)
    qa = centred_cart(km, n)
    second, _ = _second_set(shift)
    if not second:
        return qa
    c = km.astype(np.float64) - 2.0 * np.asarray(shift, dtype=np.float64)
    c = np.mod(c + n / 2.0, n) - n / 2.0
    return np.concatenate([qa, (c / n) @ recip_basis()])

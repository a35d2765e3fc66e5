"""Plain FP64 CPU oracle of the BSE hot path (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the GPU library never calls it.  It shares no code with the HIP path:
its only common ground is the seeded input generator (`bse_synth`), whose
arrays it reads.

Everything follows the paper (Vorwerk et al., "Bethe-Salpeter equation for
absorption and scattering spectroscopy: implementation in the exciting code"):

* transition energies E_a = eps_u - eps_o                         (Sec. 2.3, eq. emat)
* exchange  V_aa' = sum_G vbar_G M*_a(G) M_a'(G)                   (Sec. 4.2, eq. vrrofM,
  with the macroscopic G_Q term removed as in Sec. 4.4, eq. vbar_def)
* direct resonant  W^rr_aa' = sum_GG' w_GG'(k-k') M*_{o'o}(G) M_{u'u}(G')   (eq. wrrm)
* direct coupling  W^ra_aa' = sum_GG' w_GG'(-k-k') N*_{uo'}(G) N_{ou'}(G')  (eq. wrabar)
* A = E + 2 gx V - gc W^rr,  B = 2 gx V - gc W^ra                  (eqs. diagonalblock,
  couplingblock; (gx, gc) from the bsetype table, Appendix B)
* squared form S = (A-B)^1/2 (A+B) (A-B)^1/2, S Z = E^2 Z,
  X+Y = (A-B)^1/2 E^-1/2 Z, X-Y = (A-B)^-1/2 E^1/2 Z             (Sec. 4.3)
* TDA: A X = E X                                                   (Sec. 4.3, eq. tdaevp)
* t_l = sum_a (X+Y)*_al p_a, eps_M(w) = 1 - 2 kappa v0 sum_l |t_l|^2
  [1/(w - E_l + i eta) - 1/(w + E_l + i eta)]                      (Sec. 4.4, eqs. chir, osci)
* plain definition: eps_M(z) = 1 + 2 kappa v0 w^H (H - z Delta)^-1 w, w = [p; p],
  H = [[A, B], [B, A]]                                             (Sec. 2.3, eqs. chiofh, Hetr)

Readings of the paper taken here (each listed with its reason in the design
notes): v_G(p) = 4 pi / |G + p|^2; X - Y uses (A-B)^-1/2; the Hermitian rule
(entries with a <= a' are evaluated, the rest mirrored, the diagonal made
real); one prefactor kappa = s * Ha / (Nk * Omega) for V, W^rr and W^ra; the
spectrum prefactor 2 kappa v0 (spin 2); eta is the half width.
"""
from __future__ import annotations

import numpy as np

from . import philox

HARTREE_EV = 27.211386245988
BSE_TYPES = {"singlet": (1.0, 1.0), "triplet": (0.0, 1.0), "rpa": (1.0, 0.0), "ip": (0.0, 0.0)}


class NotPositiveDefinite(np.linalg.LinAlgError):
    pass


# ---------------------------------------------------------------- geometry
def kappa(inputs: dict) -> float:
    """Kernel prefactor s * Ha / (Nk * Omega): 1/V_c of eq. vft in eV for
    lengths in bohr, times the kernel scale s of the workload."""
    w = inputs["workload"]
    return w.kernel_scale * HARTREE_EV / (w.nk * inputs["cell_volume"])


def _gcart(inputs: dict) -> np.ndarray:
    return inputs["gvec"].astype(np.float64) * (2.0 * np.pi / inputs["alat"])


def g_of_q(inputs: dict) -> int:
    """Index of the G that carries the momentum transfer Q = G_Q + q (the G
    nearest to Q); at Q = 0 this is G = 0."""
    Q = np.asarray(inputs["workload"].q, dtype=np.float64)
    return int(np.argmin(np.sum((_gcart(inputs) - Q[None, :]) ** 2, axis=1)))


def coulomb_vbar(inputs: dict) -> np.ndarray:
    """vbar_G = 4 pi / |G + q|^2 with the G_Q term set to zero (eq. vbar_def);
    q = Q - G_Q."""
    Q = np.asarray(inputs["workload"].q, dtype=np.float64)
    G = _gcart(inputs)
    gq = g_of_q(inputs)
    q = Q - G[gq]
    p2 = np.sum((G + q[None, :]) ** 2, axis=1)
    v = np.zeros_like(p2)
    mask = np.arange(len(p2)) != gq
    v[mask] = 4.0 * np.pi / p2[mask]
    return v


def coulomb_v0(inputs: dict) -> float:
    """v at the momentum transfer, 4 pi / |Q|^2, with |Q|^2 -> 0.01 at Q = 0."""
    Q = np.asarray(inputs["workload"].q, dtype=np.float64)
    q2 = float(Q @ Q)
    return 4.0 * np.pi / (q2 if q2 > 1e-12 else 0.01)


def probe(inputs: dict) -> np.ndarray:
    """p_a = M*_a(G_Q): the plane-wave element the spectrum projects on (eq. osci)."""
    return np.conj(inputs["Mcv"][:, g_of_q(inputs)])


def q_index_of(inputs: dict, sign: int) -> np.ndarray:
    """Index into W of k - k' (sign=+1) or -k - k' (sign=-1) for every (ik, ik').
    With k = (i + s)/n (Sec. 5: shifted meshes) the difference in mesh units is
    sign (i + s) - (i' + s).  When it is integral it is a point j of the
    q-mesh (index j); otherwise it is j - 2s with j integral, a point of the
    second set, whose W entries follow the Nk of the first (index Nk + j)."""
    w = inputs["workload"]
    n = w.mesh
    kc = inputs["kcoords"].astype(np.float64) + np.asarray(w.kshift, dtype=np.float64)
    d = sign * kc[:, None, :] - kc[None, :, :]
    on_mesh = np.allclose(d, np.round(d), atol=1e-9)
    if not on_mesh:
        d = d + 2.0 * np.asarray(w.kshift, dtype=np.float64)
    j = np.mod(np.round(d).astype(np.int64), n)
    idx = (j[..., 0] * n + j[..., 1]) * n + j[..., 2]
    return idx if on_mesh else w.nk + idx


def pairs(nk: int) -> tuple[np.ndarray, np.ndarray]:
    """(ik, ik') with ik <= ik', row-major: pair p of the pair arrays."""
    return np.triu_indices(nk)


# ---------------------------------------------------------------- a1
def transition_energies(inputs: dict) -> np.ndarray:
    """E_a = eps_c[k, c] - eps_v[k, v] (+ scissor), a = (k * nv + v) * nc + c."""
    w = inputs["workload"]
    e = inputs["eps_c"][:, None, :] - inputs["eps_v"][:, :, None] + w.scissor
    return e.reshape(-1)


# ---------------------------------------------------------------- Hermitian rule
def hermitian_rule(K: np.ndarray) -> np.ndarray:
    """Keep the strict upper triangle, mirror it, take the real diagonal."""
    U = np.triu(K, 1)
    return U + U.conj().T + np.diag(K.diagonal().real)


# ---------------------------------------------------------------- a2
def exchange(inputs: dict, vbar: np.ndarray | None = None) -> np.ndarray:
    """V_aa' = sum_G vbar_G M*_a(G) M_a'(G) (eq. vrrofM with vbar)."""
    M = inputs["Mcv"]
    v = coulomb_vbar(inputs) if vbar is None else vbar
    return hermitian_rule(np.conj(M) @ (v[:, None] * M.T))


def exchange_literal(inputs: dict, vbar: np.ndarray | None = None) -> np.ndarray:
    """The same double sum written entry by entry (tiny inputs only)."""
    M = inputs["Mcv"]
    v = coulomb_vbar(inputs) if vbar is None else vbar
    n, ng = M.shape
    V = np.zeros((n, n), dtype=np.complex128)
    for a in range(n):
        for b in range(a, n):
            s = 0.0 + 0.0j
            for g in range(ng):
                s += v[g] * np.conj(M[a, g]) * M[b, g]
            V[a, b] = s
    return hermitian_rule(V)


# ---------------------------------------------------------------- a3 / a4
def _place_blocks(nk: int, nvnc: int, ik, jk, blocks) -> np.ndarray:
    K = np.zeros((nk, nvnc, nk, nvnc), dtype=np.complex128)
    K[ik, :, jk, :] = blocks
    return K.reshape(nk * nvnc, nk * nvnc)


def mcc(inputs: dict, ps) -> np.ndarray:
    """M_{u u'}(G') of the pairs ps: the stored array, or the values drawn from
    the workload's key and envelope (counter-based generator, oracle.philox)."""
    if inputs.get("Mcc") is not None:
        return inputs["Mcc"][ps]
    w = inputs["workload"]
    return philox.mcc_pairs(inputs["mcc_key"], inputs["mcc_env"], np.atleast_1d(ps), w.nc)


def direct_blocks(inputs: dict, which: str, sel: np.ndarray | None = None) -> np.ndarray:
    """(nv*nc x nv*nc) blocks of W^rr ("rr") or W^ra ("ra") for the pairs `sel`
    (all pairs by default), contracted per momentum-transfer class:
      rr: T = M*_vv W(k-k'),   block[(v,c),(v',c')] = sum_G' T[v,v',G'] Mcc[c,c',G']
      ra: T = N*_cv W(-k-k'),  block[(v,c),(v',c')] = sum_G' T[c,v',G'] Nvc[v,c',G']"""
    w = inputs["workload"]
    nk, nv, nc, ng = w.nk, w.nv, w.nc, w.ng
    ik, jk = pairs(nk)
    if sel is None:
        sel = np.arange(len(ik))
    qi = q_index_of(inputs, +1 if which == "rr" else -1)[ik[sel], jk[sel]]
    out = np.empty((len(sel), nv, nc, nv, nc), dtype=np.complex128)
    Wq = inputs["W"]
    if which == "rr":
        left, right = inputs["Mvv"], (lambda ps: mcc(inputs, ps))
    else:
        left, right = inputs["Ncv"], (lambda ps: inputs["Nvc"][ps])
    for q in np.unique(qi):
        m = np.nonzero(qi == q)[0]
        ps = sel[m]
        L = np.conj(left[ps])
        T = (L.reshape(-1, ng) @ Wq[q]).reshape(L.shape)
        R = right(ps)
        if which == "rr":
            # T[p, v, v', G'], R[p, c, c', G'] -> [p, v, c, v', c']
            out[m] = np.einsum("pabg,pcdg->pacbd", T, R)
        else:
            # T[p, c, v', G'], R[p, v, c', G'] -> [p, v, c, v', c']
            out[m] = np.einsum("pcbg,padg->pacbd", T, R)
    return out


def direct(inputs: dict, which: str) -> np.ndarray:
    w = inputs["workload"]
    ik, jk = pairs(w.nk)
    blk = direct_blocks(inputs, which).reshape(len(ik), w.nv * w.nc, w.nv * w.nc)
    return hermitian_rule(_place_blocks(w.nk, w.nv * w.nc, ik, jk, blk))


def direct_literal(inputs: dict, which: str) -> np.ndarray:
    """W^rr / W^ra as the literal double sum over (G, G') for every a <= a'
    (tiny inputs only)."""
    w = inputs["workload"]
    nk, nv, nc = w.nk, w.nv, w.nc
    qmat = q_index_of(inputs, +1 if which == "rr" else -1)
    n = w.n
    K = np.zeros((n, n), dtype=np.complex128)
    pid = -np.ones((nk, nk), dtype=np.int64)
    ik, jk = pairs(nk)
    pid[ik, jk] = np.arange(len(ik))
    for a in range(n):
        k1, r = divmod(a, nv * nc)
        o, u = divmod(r, nc)
        for b in range(a, n):
            k2, r2 = divmod(b, nv * nc)
            o2, u2 = divmod(r2, nc)
            p = pid[k1, k2]
            Wq = inputs["W"][qmat[k1, k2]]
            if which == "rr":
                x = np.conj(inputs["Mvv"][p, o, o2])
                y = mcc(inputs, [p])[0, u, u2]
            else:
                x = np.conj(inputs["Ncv"][p, u, o2])
                y = inputs["Nvc"][p, o, u2]
            K[a, b] = np.sum(x[:, None] * Wq * y[None, :])
    return hermitian_rule(K)


# ---------------------------------------------------------------- a5
def assemble(inputs: dict, bse_type: str = "singlet", literal: bool = False,
             vbar: np.ndarray | None = None, coupling: str | None = None):
    """A and B of eqs. diagonalblock / couplingblock (B is None in the TDA)."""
    w = inputs["workload"]
    coupling = coupling or w.coupling
    gx, gc = BSE_TYPES[bse_type]
    kap = kappa(inputs)
    E = transition_energies(inputs)
    V = (exchange_literal if literal else exchange)(inputs, vbar)
    Wrr = (direct_literal if literal else direct)(inputs, "rr")
    A = np.diag(E).astype(np.complex128) + kap * (2.0 * gx * V - gc * Wrr)
    if coupling == "tda":
        return A, None
    Wra = (direct_literal if literal else direct)(inputs, "ra")
    B = kap * (2.0 * gx * V - gc * Wra)
    return A, B


def kernel_blocks(inputs: dict, sel: np.ndarray, bse_type: str = "singlet"):
    """Blocks (ik, ik') of A+B and A-B (full) or A (TDA) for the pairs `sel`,
    before the Hermitian rule (diagonal pairs hold every entry of the block)."""
    w = inputs["workload"]
    nv, nc, nvnc = w.nv, w.nc, w.nv * w.nc
    gx, gc = BSE_TYPES[bse_type]
    kap = kappa(inputs)
    ik, jk = pairs(w.nk)
    M = inputs["Mcv"].reshape(w.nk, nvnc, w.ng)
    v = coulomb_vbar(inputs)
    V = np.einsum("pag,g,pbg->pab", np.conj(M[ik[sel]]), v, M[jk[sel]])
    Wrr = direct_blocks(inputs, "rr", sel).reshape(len(sel), nvnc, nvnc)
    E = transition_energies(inputs).reshape(w.nk, nvnc)
    Ed = np.zeros((len(sel), nvnc, nvnc), dtype=np.complex128)
    dg = ik[sel] == jk[sel]
    Ed[dg] = np.einsum("pa,ab->pab", E[ik[sel][dg]], np.eye(nvnc))
    if w.coupling == "tda":
        return Ed + kap * (2.0 * gx * V - gc * Wrr), None
    Wra = direct_blocks(inputs, "ra", sel).reshape(len(sel), nvnc, nvnc)
    ApB = Ed + kap * (4.0 * gx * V - gc * (Wrr + Wra))
    AmB = Ed - kap * gc * (Wrr - Wra)
    return ApB, AmB


# ---------------------------------------------------------------- a6..a10
def _herm(X: np.ndarray) -> np.ndarray:
    return 0.5 * (X + X.conj().T)


def solve_full(A: np.ndarray, B: np.ndarray):
    """Squared form of Sec. 4.3 with the literal square root of A - B.
    Returns E (ascending), X+Y and X-Y (columns are eigenvectors)."""
    d, U = np.linalg.eigh(_herm(A - B))
    if d[0] <= 0.0:
        raise NotPositiveDefinite("A - B is not positive definite")
    sd = np.sqrt(d)
    R = (U * sd[None, :]) @ U.conj().T
    Rinv = (U / sd[None, :]) @ U.conj().T
    S = _herm(R @ (A + B) @ R)
    mu, Z = np.linalg.eigh(S)
    if mu[0] <= 0.0:
        raise NotPositiveDefinite("A + B is not positive definite")
    E = np.sqrt(mu)
    XpY = (R @ Z) / np.sqrt(E)[None, :]
    XmY = (Rinv @ Z) * np.sqrt(E)[None, :]
    return E, XpY, XmY


def solve_tda(A: np.ndarray):
    """Hermitian eigenproblem A X = E X (eq. tdaevp)."""
    E, X = np.linalg.eigh(_herm(A))
    return E, X


def solve(A, B):
    if B is None:
        E, X = solve_tda(A)
        return E, X, X
    return solve_full(A, B)


# ---------------------------------------------------------------- a11 / a12
def oscillator(XpY: np.ndarray, p: np.ndarray) -> np.ndarray:
    """|t_l|^2 with t_l = sum_a (X+Y)*_al p_a (eq. osci, 1/V_c moved into the prefactor)."""
    return np.abs(XpY.conj().T @ p) ** 2


def spectrum(E: np.ndarray, t2: np.ndarray, omega: np.ndarray, eta: float, pref: float):
    """eps_M(w) = 1 - pref * sum_l t2_l [1/(w - E_l + i eta) - 1/(w + E_l + i eta)]
    (eq. chir inserted in eps_M = 1 - v Pbar)."""
    z = omega[:, None] + 1j * eta
    return 1.0 - pref * np.sum(t2[None, :] * (1.0 / (z - E[None, :]) - 1.0 / (z + E[None, :])),
                               axis=1)


def spectrum_prefactor(inputs: dict) -> float:
    """2 kappa v0: spin factor 2, 1/V_c and v(Q) of eps_M = 1 - v(Q) Pbar."""
    return 2.0 * kappa(inputs) * coulomb_v0(inputs)


def resolvent_spectrum(A, B, p, omega, eta, pref):
    """Plain definition: eps_M(z) = 1 + pref * w^H (H - z Delta)^-1 w with
    H = [[A, B], [B, A]], Delta = diag(1, -1), w = [p; p], z = w + i eta."""
    n = A.shape[0]
    Bm = np.zeros_like(A) if B is None else B
    H = np.block([[A, Bm], [Bm, A]])
    D = np.concatenate([np.ones(n), -np.ones(n)])
    wv = np.concatenate([p, p])
    out = np.empty(len(omega), dtype=np.complex128)
    for i, om in enumerate(omega):
        z = om + 1j * eta
        x = np.linalg.solve(H - z * np.diag(D), wv)
        out[i] = 1.0 + pref * np.vdot(wv, x)
    return out


def brute_force_2n(A, B):
    """Eigenvalues of Delta H (the 2N non-Hermitian form, eq. gevpbse), sorted."""
    n = A.shape[0]
    Bm = np.zeros_like(A) if B is None else B
    H = np.block([[A, Bm], [Bm, A]])
    D = np.concatenate([np.ones(n), -np.ones(n)])
    ev = np.linalg.eigvals(D[:, None] * H)
    return np.sort(ev.real), ev


def run(inputs: dict, bse_type: str = "singlet"):
    """Whole path: assemble, solve, spectrum.  Returns a dict of results."""
    A, B = assemble(inputs, bse_type)
    E, XpY, XmY = solve(A, B)
    p = probe(inputs)
    t2 = oscillator(XpY, p)
    pref = spectrum_prefactor(inputs)
    w = inputs["workload"]
    eps = spectrum(E, t2, inputs["omega"], w.eta, pref)
    return {"A": A, "B": B, "E": E, "XpY": XpY, "XmY": XmY, "t2": t2, "eps": eps,
            "pref": pref, "p": p}

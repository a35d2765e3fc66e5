"""Workload table: seeded synthetic BSE problems shaped like the paper's runs.

Each workload fixes the index spaces (k-mesh, band window, plane-wave shell),
the distributions the generator draws from, the frequency grid and the
broadening.  Sizes follow the paper's applications (Sec. 5: 8x8x8 shifted
meshes with 4+12 bands for LiF/Si, 0.1 eV broadening for Si, core states for
the F K-edge); the inputs themselves are synthetic because the paper's DFT
wavefunctions are not available.

kernel_scale (s) multiplies the kernel prefactor kappa = s * Ha / (Nk * Omega).
The bare synthetic kernel is a random matrix that would destroy the positive
definiteness of A-B and A+B that the squared form needs (Sec. 4.3), so s is the
largest power of two for which A-B, A+B (full) or A (TDA) keep every eigenvalue
above a tenth of the smallest transition energy.  The values below were found
by `oracle/calibrate_scale.py` and are re-checked by the CPU tests.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace


@dataclass(frozen=True)
class Workload:
    name: str
    mesh: int                 # k-mesh is mesh x mesh x mesh (Gamma-centred unless kshift)
    nv: int                   # occupied (valence or core) bands
    nc: int                   # unoccupied bands
    ng: int                   # plane waves (closed shell)
    coupling: str             # "tda" or "full"
    nw: int                   # frequency points
    wmin: float               # eV
    wmax: float               # eV
    eta: float                # Lorentzian half width (eV) = broadening FWHM / 2
    seed: int
    kernel_scale: float
    q: tuple = (0.0, 0.0, 0.0)   # momentum transfer (bohr^-1)
    eps_v_range: tuple = (-3.0, 0.0)
    eps_c_range: tuple = (1.0, 5.0)
    core_level: float | None = None   # flat core levels (eV) instead of eps_v draws
    mcv_gauss_width: float | None = None  # Gaussian |G+Q| envelope of Mcv (bohr^-1)
    mcc_generated: bool = False  # Mcc given by a key and an envelope, drawn where used
    scissor: float = 0.0
    kshift: tuple = (0.0, 0.0, 0.0)  # k = (i + kshift) / mesh along b1, b2, b3
    orbitals: int = 0         # > 0: pair elements come from synthetic orbitals expanded in
                              # this many plane waves (a closed shell), not drawn directly
    note: str = ""

    @property
    def nk(self) -> int:
        return self.mesh ** 3

    @property
    def n(self) -> int:
        return self.nk * self.nv * self.nc

    @property
    def npairs(self) -> int:
        return self.nk * (self.nk + 1) // 2


WORKLOADS: dict[str, Workload] = {}


def _add(w: Workload) -> Workload:
    WORKLOADS[w.name] = w
    return w


# Small TDA problem at Q = 0 (N = 384): the size the oracle finishes in seconds.
TDA_N384 = _add(Workload(
    name="tda_q0_k4_v2c3_g59", mesh=4, nv=2, nc=3, ng=59, coupling="tda",
    nw=2000, wmin=0.0, wmax=10.0, eta=0.05, seed=0, kernel_scale=0.125,
    note="Plain TDA BSE at Q=0, N=384 transitions, 59 plane waves"))

# Full (non-TDA) problem at Q = 0 with N = 6144 (2N = 12288): the headline size.
FULL_N6144 = _add(Workload(
    name="full_q0_k8_v3c4_g113", mesh=8, nv=3, nc=4, ng=113, coupling="full",
    nw=4000, wmin=0.0, wmax=10.0, eta=0.05, seed=1, kernel_scale=0.25,
    note="Full BSE at Q=0, N=6144 transitions, 113 plane waves"))

# Core-level (x-ray) TDA problem: two flat core levels at -400 eV, 32 conduction
# bands, N = 32768, 137 plane waves, Mcv with a narrow Gaussian G-profile (a
# localised core state), 8000 frequencies within 30 eV of the edge.  Its Mcc
# would take 295 GB (131 328 pairs x 32 x 32 x 137), so it is given by a key and
# an envelope and drawn where it is used.  With core transition energies near
# 400 eV every kernel scale keeps A positive definite; s = 1 is the unscaled
# prefactor 1/V_c.
CORE_N32768 = _add(Workload(
    name="core_tda_k8_c2c32_g137", mesh=8, nv=2, nc=32, ng=137, coupling="tda",
    nw=8000, wmin=371.0, wmax=431.0, eta=0.05, seed=4, kernel_scale=1.0,
    core_level=-400.0, mcv_gauss_width=0.5, mcc_generated=True,
    note="Core-level TDA BSE, N=32768 transitions, 137 plane waves, Mcc drawn in place"))

# Tiny problems used by the CPU pins and the GPU parity tests (several tiles
# and ragged tails).
TINY = {
    "tiny_tda": _add(Workload(name="tiny_tda_k2_v2c2_g9", mesh=2, nv=2, nc=2, ng=9,
                              coupling="tda", nw=200, wmin=0.0, wmax=10.0, eta=0.05,
                              seed=11, kernel_scale=0.0625)),
    "tiny_full": _add(Workload(name="tiny_full_k2_v2c3_g15", mesh=2, nv=2, nc=3, ng=15,
                               coupling="full", nw=200, wmin=0.0, wmax=10.0, eta=0.05,
                               seed=12, kernel_scale=0.03125)),
    "small_full": _add(Workload(name="small_full_k3_v3c4_g27", mesh=3, nv=3, nc=4, ng=27,
                                coupling="full", nw=500, wmin=0.0, wmax=10.0, eta=0.05,
                                seed=13, kernel_scale=0.0625)),
    # shifted meshes (a generic offset as in the paper's runs): -k-k' falls on a
    # second q-set, so W is given on both sets (nq = 2 Nk)
    "tiny_full_shift": _add(Workload(name="tiny_full_k2s_v2c3_g15", mesh=2, nv=2, nc=3, ng=15,
                                     coupling="full", nw=200, wmin=0.0, wmax=10.0, eta=0.05,
                                     seed=17, kernel_scale=0.03125,
                                     kshift=(0.097, 0.273, 0.493))),
    "small_full_shift": _add(Workload(name="small_full_k3s_v3c4_g27", mesh=3, nv=3, nc=4,
                                      ng=27, coupling="full", nw=500, wmin=0.0, wmax=10.0,
                                      eta=0.05, seed=18, kernel_scale=0.03125,
                                      kshift=(0.097, 0.273, 0.493))),
    # half-step offset: -k-k' lands back on the unshifted q-mesh (nq = Nk)
    "tiny_full_half": _add(Workload(name="tiny_full_k2h_v2c3_g15", mesh=2, nv=2, nc=3, ng=15,
                                    coupling="full", nw=200, wmin=0.0, wmax=10.0, eta=0.05,
                                    seed=19, kernel_scale=0.03125, kshift=(0.5, 0.5, 0.5))),
    "mid_full": _add(Workload(name="mid_full_k4_v3c4_g59", mesh=4, nv=3, nc=4, ng=59,
                              coupling="full", nw=1000, wmin=0.0, wmax=10.0, eta=0.05,
                              seed=14, kernel_scale=0.0625)),
    # N_G = 113 (the benchmark's) and 51: one and three plane waves past a
    # multiple of 16, one and three past a multiple of 4
    "small_full_g113": _add(Workload(name="small_full_k3_v3c4_g113", mesh=3, nv=3, nc=4, ng=113,
                                     coupling="full", nw=500, wmin=0.0, wmax=10.0, eta=0.05,
                                     seed=41, kernel_scale=0.03125)),
    "tiny_full_g51": _add(Workload(name="tiny_full_k2_v3c4_g51", mesh=2, nv=3, nc=4, ng=51,
                                   coupling="full", nw=200, wmin=0.0, wmax=10.0, eta=0.05,
                                   seed=42, kernel_scale=0.015625)),
    # the core-level structure (flat core levels, Gaussian Mcv, Mcc drawn in
    # place) at sizes the oracle solves whole
    "tiny_core": _add(Workload(name="tiny_core_k2_c2c6_g27", mesh=2, nv=2, nc=6, ng=27,
                               coupling="tda", nw=300, wmin=371.0, wmax=431.0, eta=0.05,
                               seed=15, kernel_scale=1.0, core_level=-400.0,
                               mcv_gauss_width=0.5, mcc_generated=True)),
    "tiny_core_g137": _add(Workload(name="tiny_core_k2_c2c4_g137", mesh=2, nv=2, nc=4, ng=137,
                                    coupling="tda", nw=300, wmin=371.0, wmax=431.0, eta=0.05,
                                    seed=17, kernel_scale=1.0, core_level=-400.0,
                                    mcv_gauss_width=0.5, mcc_generated=True)),
    "mid_core": _add(Workload(name="mid_core_k4_c2c8_g59", mesh=4, nv=2, nc=8, ng=59,
                              coupling="tda", nw=1000, wmin=371.0, wmax=431.0, eta=0.05,
                              seed=16, kernel_scale=1.0, core_level=-400.0,
                              mcv_gauss_width=0.5, mcc_generated=True)),
    # pair elements from synthetic orbitals (plane-wave coefficients on a
    # sphere of K-vectors), formed where they are used
    "tiny_orb": _add(Workload(name="tiny_orb_k2_v2c3_g15_o27", mesh=2, nv=2, nc=3, ng=15,
                              coupling="full", nw=200, wmin=0.0, wmax=10.0, eta=0.05, seed=31,
                              kernel_scale=0.0625, orbitals=27)),
    "small_orb": _add(Workload(name="small_orb_k3_v3c4_g27_o51", mesh=3, nv=3, nc=4, ng=27,
                               coupling="full", nw=500, wmin=0.0, wmax=10.0, eta=0.05, seed=32,
                               kernel_scale=0.125, orbitals=51)),
    "mid_orb_tda": _add(Workload(name="mid_orb_tda_k4_v2c3_g59_o89", mesh=4, nv=2, nc=3, ng=59,
                                 coupling="tda", nw=1000, wmin=0.0, wmax=10.0, eta=0.05,
                                 seed=33, kernel_scale=0.5, orbitals=89)),
}




# The benchmark workload's shape with its pair elements formed from orbitals
# (113 plane waves per orbital), for the on-device generation of the elements.
FULL_ORB = _add(Workload(
    name="full_orb_k8_v3c4_g113_o113", mesh=8, nv=3, nc=4, ng=113, coupling="full",
    nw=4000, wmin=0.0, wmax=10.0, eta=0.05, seed=34, kernel_scale=1.0, orbitals=113,
    note="Full BSE at Q=0, N=6144, pair elements from synthetic orbitals"))


@dataclass(frozen=True)
class BatchWorkload:
    """Many momentum transfers Q solved as one batch: W(q) and the pair
    elements are shared (drawn once for the widest band window and sliced),
    energies and M_cv are drawn per Q."""
    name: str
    members: tuple            # Workload per Q (own nv, nc, q, seed)
    master: Workload          # widest band window; seed of the shared arrays

    @property
    def sizes(self) -> list:
        return [m.n for m in self.members]


def _batch(name, mesh, ng, nq, qmax, nvs, ncs, seed, kernel_scale, nw, wmax, coupling="full"):
    members = []
    for i in range(nq):
        nv, nc = nvs[i % len(nvs)], ncs[i % len(ncs)]
        q = (qmax * i / (nq - 1), 0.0, 0.0) if nq > 1 else (0.0, 0.0, 0.0)
        members.append(Workload(name=f"{name}_q{i}", mesh=mesh, nv=nv, nc=nc, ng=ng,
                                coupling=coupling, nw=nw, wmin=0.0, wmax=wmax, eta=0.05,
                                seed=seed + 101 + i, kernel_scale=kernel_scale, q=q))
    master = Workload(name=f"{name}_master", mesh=mesh, nv=max(nvs), nc=max(ncs), ng=ng,
                      coupling=coupling, nw=nw, wmin=0.0, wmax=wmax, eta=0.05, seed=seed,
                      kernel_scale=kernel_scale)
    return BatchWorkload(name=name, members=tuple(members), master=master)


BATCHES: dict[str, BatchWorkload] = {}
# 16 momentum transfers Q = (0.1 i, 0, 0) bohr^-1 along Gamma-X, 6x6x6 mesh,
# N_v = 2 + (i mod 3), N_c = 3 + (i mod 4): N from 1296 to 5184
BATCHES["batch16_k6_g89"] = _batch("batch16_k6_g89", mesh=6, ng=89, nq=16, qmax=1.5,
                                   nvs=(2, 3, 4), ncs=(3, 4, 5, 6), seed=3,
                                   kernel_scale=0.125, nw=2000, wmax=10.0)
# small batch for the parity tests (uneven sizes, several tiles, finite Q)
BATCHES["batch4_k2_g15"] = _batch("batch4_k2_g15", mesh=2, ng=15, nq=4, qmax=1.5,
                                  nvs=(1, 2, 3), ncs=(2, 3), seed=21, kernel_scale=0.015625,
                                  nw=300, wmax=10.0)
BATCHES["batch3_k3_g27"] = _batch("batch3_k3_g27", mesh=3, ng=27, nq=3, qmax=0.9,
                                  nvs=(2, 3, 2), ncs=(3, 4, 2), seed=22, kernel_scale=0.03125,
                                  nw=300, wmax=10.0)
# more problems than one batched launch takes (16): the batched stages run in two groups
BATCHES["batch18_k2_g15"] = _batch("batch18_k2_g15", mesh=2, ng=15, nq=18, qmax=1.5,
                                   nvs=(1, 2, 3), ncs=(2, 3), seed=23, kernel_scale=0.015625,
                                   nw=200, wmax=10.0)
# the smallest orders (N = 1, 2, 6: no Householder step, a single one, one panel)
BATCHES["batch3_k1_g9"] = _batch("batch3_k1_g9", mesh=1, ng=9, nq=3, qmax=0.5, nvs=(1, 2, 2),
                                 ncs=(1, 1, 3), seed=25, kernel_scale=0.004, nw=100, wmax=10.0)
# Tamm-Dancoff members (no Cholesky factorisation, no coupling block)
BATCHES["batch5_tda_k2_g15"] = _batch("batch5_tda_k2_g15", mesh=2, ng=15, nq=5, qmax=1.2,
                                      nvs=(1, 2, 3), ncs=(2, 3), seed=24, kernel_scale=0.015625,
                                      nw=200, wmax=10.0, coupling="tda")


def get(name: str) -> Workload:
    return WORKLOADS[name]


def with_(w: Workload, **kw) -> Workload:
    return replace(w, **kw)

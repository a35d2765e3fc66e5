"""GPU parity of the optical-limit observables through the C ABI: transition
coefficients (eq. tlambdai), the dielectric tensor (eq. epsmij), the loss
function and S(Q, w) (eq. Lofeps), against the FP64 oracle.

Tolerances:
  kernel on the same inputs (t, eps^ij, loss, S)   1e-12 of the largest value
  end to end (GPU solve + tensor vs the oracle)    1e-10 of max|eps - 1|
The benchmark's size (N = 6144) is covered in test_gpu_fullsize.py.
"""
import numpy as np
import pytest

from oracle import observables as X
from tests._cache import inputs, oracle_run

pytestmark = pytest.mark.gpu


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("n,nprobe", [(1, 1), (37, 2), (300, 3), (1001, 4), (2056, 3)])
def test_transitions_kernel_ragged_sizes(n, nprobe):
    """Random X and probes (the kernel does not need eigenvectors): n below,
    across and not a multiple of the 8-column and 256-row tiles; leading
    dimensions larger than n."""
    torch = _torch()
    from paper_1904_05575_amd import _lib as L
    print(f"[gpu] transitions n={n} nprobe={nprobe}", flush=True)
    rng = np.random.default_rng(n)
    ldx, ldp, ldt = n + 3, n + 5, n + 1
    Xh = rng.standard_normal((ldx, n)) + 1j * rng.standard_normal((ldx, n))  # [col][row]
    Xh = Xh.T.copy()  # rows: columns of X, padded to ldx
    Ph = rng.standard_normal((nprobe, ldp)) + 1j * rng.standard_normal((nprobe, ldp))
    Xd = torch.from_numpy(Xh.reshape(-1)).cuda()
    Pd = torch.from_numpy(Ph.reshape(-1)).cuda()
    td = torch.zeros(nprobe * ldt, dtype=torch.complex128, device="cuda")
    L.bse_transitions(n, Xd.data_ptr(), ldx, nprobe, Pd.data_ptr(), ldp, td.data_ptr(), ldt,
                      torch.cuda.current_stream().cuda_stream)
    got = td.cpu().numpy().reshape(nprobe, ldt)[:, :n].T      # [l, i]
    Xm = Xh.reshape(n, ldx)[:, :n].T                           # X[a, l]
    D = Ph[:, :n].T.conj()                                     # probe = conj(D)
    ref = X.transition_coefficients(Xm, D)
    assert _rel(got, ref) < 1e-12
    assert np.all(td.cpu().numpy().reshape(nprobe, ldt)[:, n:] == 0)  # padding untouched


@pytest.mark.parametrize("nd,nw", [(1, 5), (2, 257), (3, 4001)])
def test_dielectric_tensor_and_loss_kernels(nd, nw):
    torch = _torch()
    from paper_1904_05575_amd import _lib as L
    print(f"[gpu] tensor nd={nd} nw={nw}", flush=True)
    rng = np.random.default_rng(nd)
    n = 777
    E = np.sort(rng.uniform(0.5, 6.0, n))
    ldt = n + 2
    T = rng.standard_normal((nd, ldt)) + 1j * rng.standard_normal((nd, ldt))
    om = np.linspace(0.0, 8.0, nw)
    eta, pref = 0.05, 0.3
    s = torch.cuda.current_stream().cuda_stream
    Ed, Td, Od = (torch.from_numpy(a.reshape(-1)).cuda() for a in (E, T, om))
    eps = torch.empty(nw * nd * nd, dtype=torch.complex128, device="cuda")
    L.bse_dielectric_tensor(n, Ed.data_ptr(), nd, Td.data_ptr(), ldt, pref, eta, nw,
                            Od.data_ptr(), eps.data_ptr(), s)
    got = eps.cpu().numpy().reshape(nw, nd, nd)
    ref = X.dielectric_tensor(E, T[:, :n].T, om, eta, pref)
    assert _rel(got, ref) < 1e-12
    for a in range(nd):
        loss = torch.empty(nw, dtype=torch.float64, device="cuda")
        sqw = torch.empty(nw, dtype=torch.float64, device="cuda")
        L.bse_loss(nw, eps.data_ptr() + 16 * a * (nd + 1), nd * nd, 0.7, loss.data_ptr(),
                   sqw.data_ptr(), s)
        assert _rel(loss.cpu().numpy(), X.loss_function(ref[:, a, a])) < 1e-12
        assert _rel(sqw.cpu().numpy(), X.dynamic_structure_factor(ref[:, a, a], 1.0 / 0.7)) < 1e-12
    loss = torch.empty(nw, dtype=torch.float64, device="cuda")
    L.bse_loss(nw, eps.data_ptr(), 1, 1.0, loss.data_ptr(), 0, s)  # no S requested
    flat = ref.reshape(-1)[:nw]
    assert _rel(loss.cpu().numpy(), X.loss_function(flat)) < 1e-12


@pytest.mark.parametrize("name", ["tiny_tda_k2_v2c2_g9", "tiny_full_k2_v2c3_g15",
                                  "small_full_k3_v3c4_g27", "tda_q0_k4_v2c3_g59"])
def test_observables_end_to_end_against_the_oracle(name):
    """GPU build + solve (vectors) + transitions + tensor + loss vs the
    oracle's whole path; the tensor and the loss are gauge free."""
    _torch()
    from paper_1904_05575_amd.bse import Problem
    print(f"[gpu] observables {name}", flush=True)
    d, r = inputs(name), oracle_run(name)
    P = Problem(d)
    H0, H1 = P.build()
    E, XpY, _ = P.solve(H0, H1, vectors=True, probe=False)
    t = P.transitions(XpY)
    eps = P.dielectric_tensor(E, t)
    loss = [P.loss(eps, diag=a) for a in range(3)]
    P.check_info()
    # the kernels on the GPU's own E and X+Y
    XpYh = XpY.T.cpu().numpy()
    th = t.cpu().numpy().T
    assert _rel(th, X.transition_coefficients(XpYh, d["Dcv"])) < 1e-12
    epsh = eps.cpu().numpy()
    om, eta, pref = d["omega"], d["workload"].eta, X.tensor_prefactor(d)
    assert _rel(epsh, X.dielectric_tensor(E.cpu().numpy(), th, om, eta, pref)) < 1e-12
    # against the oracle's whole path
    ref = X.dielectric_tensor(r["E"], X.transition_coefficients(r["XpY"], d["Dcv"]), om, eta,
                              pref)
    dev = ref - np.eye(3)[None]
    assert np.abs(epsh - ref).max() < 1e-10 * np.abs(dev).max()
    from oracle.bse_oracle import coulomb_v0
    for a in range(3):
        L_, S = (v.cpu().numpy() for v in loss[a])
        assert _rel(L_, X.loss_function(ref[:, a, a])) < 1e-9
        assert _rel(S, X.dynamic_structure_factor(ref[:, a, a], coulomb_v0(d))) < 1e-9

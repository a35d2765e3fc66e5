"""Host-side checks of the C-ABI library (no GPU needed): every function that
include/bse.h declares is exported, workspace sizing and argument checks."""
import ctypes
import os
import re

import pytest

from paper_1904_05575_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "bse.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bse_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libbse.so is not built (run `python -m paper_1904_05575_amd.build`)")
    return L.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert set(L.EXPORTS) <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def _desc(**kw):
    d = dict(nk=8, nv=2, nc=3, ng=15, coupling=L.BSE_FULL, type=L.BSE_SINGLET,
             prec=L.BSE_PREC_FP64, split_terms=0, kappa=0.01, scissor=0.0, ld=48)
    d.update(kw)
    return L.BseDesc(**d)


def test_workspace_sizes(lib):
    assert L.bse_workspace_size(_desc(), L.BSE_STAGE_BUILD) > 0
    assert L.bse_workspace_size(_desc(), L.BSE_STAGE_SOLVE) > 0
    tda = L.bse_workspace_size(_desc(coupling=L.BSE_TDA), L.BSE_STAGE_BUILD)
    assert 0 < tda < L.bse_workspace_size(_desc(), L.BSE_STAGE_BUILD)
    for bad in (dict(nk=0), dict(ld=47), dict(coupling=7), dict(type=9), dict(prec=5),
                dict(kappa=float("nan"))):
        assert L.bse_workspace_size(_desc(**bad), L.BSE_STAGE_BUILD) == 0, bad
    assert L.bse_workspace_size(_desc(), 9) == 0


def test_argument_errors_are_reported_without_launching(lib):
    d = _desc()
    inp = L.BseInputs()
    with pytest.raises(L.BseError, match="BSE_ERR_ARG"):
        L.bse_build(d, inp, 1, 1, 1, 1 << 30, 1, 0)       # null input pointers
    full = L.BseInputs(eps_v=1, eps_c=1, Mcv=1, Mvv=1, Mcc=1, Ncv=1, Nvc=1, W=1, vbar=1,
                       qmap=1, qramap=1, nq=17, reserved=0)
    with pytest.raises(L.BseError, match="BSE_ERR_ARG"):          # the precision form's W
        L.bse_build(_desc(prec=L.BSE_PREC_BF16X3), full, 1, 1, 1, 1 << 40, 1, 0)  # split: nq <= 2 nk
    with pytest.raises(L.BseError, match="BSE_ERR_WORKSPACE"):     # FP64 accepts nq > nk
        L.bse_build(d, full, 1, 1, 1, 16, 1, 0)
    drawn = L.BseInputs(eps_v=1, eps_c=1, Mcv=1, Mvv=1, Mcc=None, Ncv=1, Nvc=1, W=1, vbar=1,
                        qmap=1, qramap=1, nq=9, reserved=0, mcc_env=None, mcc_key=5)
    with pytest.raises(L.BseError, match="BSE_ERR_ARG"):          # no Mcc and no envelope
        L.bse_build(d, drawn, 1, 1, 1, 1 << 40, 1, 0)
    drawn.mcc_env = 1
    with pytest.raises(L.BseError, match="BSE_ERR_ARG"):          # drawn Mcc: nv^2 <= 16
        L.bse_build(_desc(nv=5, ld=120), drawn, 1, 1, 1, 1 << 40, 1, 0)
    with pytest.raises(L.BseError, match="BSE_ERR_ARG"):
        L.bse_solve(d, 1, 0, 1, 0, 0, 48, 0, 0, 1, 1 << 30, 1, 0)   # full needs H1
    with pytest.raises(L.BseError, match="BSE_ERR_ARG"):
        L.bse_solve(d, 1, 1, 1, 0, 2, 48, 0, 0, 1, 1 << 40, 1, 0)   # X-Y needs X+Y
    with pytest.raises(L.BseError, match="BSE_ERR_ARG"):
        L.bse_solve(d, 1, 1, 1, 2, 2, 48, 0, 0, 1, 1 << 40, 1, 0)   # X-Y in its own buffer
    with pytest.raises(L.BseError, match="BSE_ERR_WORKSPACE"):
        L.bse_solve(d, 1, 1, 1, 1, 0, 48, 0, 0, 1, 16, 1, 0)
    with pytest.raises(L.BseError, match="BSE_ERR_ARG"):
        L.bse_spectrum(10, 1, 1, 1.0, 0.0, 5, 1, 1, 0)      # eta must be > 0
    with pytest.raises(L.BseError, match="BSE_ERR_ARG"):
        L.bse_oscillator(10, 1, 5, 1, 1, 0)                 # ldx < n
    for bad in (dict(nprobe=0), dict(nprobe=5), dict(ldp=9), dict(ldt=9), dict(ldx=9),
                dict(n=0), dict(probe=0)):
        a = dict(n=10, XpY=1, ldx=10, nprobe=3, probe=1, ldp=10, t=1, ldt=10, stream=0)
        a.update(bad)
        with pytest.raises(L.BseError, match="BSE_ERR_ARG"):
            L.bse_transitions(**a)
    for bad in (dict(nd=0), dict(nd=4), dict(ldt=9), dict(eta=0.0), dict(nw=0),
                dict(pref=float("nan"))):
        a = dict(n=10, E=1, nd=3, t=1, ldt=10, pref=1.0, eta=0.1, nw=5, omega=1, eps=1, stream=0)
        a.update(bad)
        with pytest.raises(L.BseError, match="BSE_ERR_ARG"):
            L.bse_dielectric_tensor(**a)
    for bad in (dict(nw=0), dict(inc=0), dict(loss=0), dict(vinv=0.0), dict(vinv=float("inf"))):
        a = dict(nw=5, eps=1, inc=1, vinv=1.0, loss=1, sqw=1, stream=0)
        a.update(bad)
        with pytest.raises(L.BseError, match="BSE_ERR_ARG"):
            L.bse_loss(**a)
    sd = dict(nk=8, nv=2, nc=3, ng=15, inv_vc=0.01, units_per_hartree=27.2)
    assert L.bse_screening_workspace_size(L.BseScreenDesc(**sd)) == 2 * 8 * 8 * 2 * 3 * 8
    for bad in (dict(ng=0), dict(ng=513), dict(nk=0), dict(nv=0), dict(inv_vc=-1.0),
                dict(units_per_hartree=float("nan"))):
        d2 = L.BseScreenDesc(**{**sd, **bad})
        assert L.bse_screening_workspace_size(d2) == 0, bad
        with pytest.raises(L.BseError, match="BSE_ERR_ARG"):
            L.bse_screening(d2, 1, 1, 1, 1, 1, 1, 1, 1, 1 << 30, 1, 0)
    with pytest.raises(L.BseError, match="BSE_ERR_ARG"):
        L.bse_screening(L.BseScreenDesc(**sd), 1, 1, 0, 1, 1, 1, 1, 1, 1 << 30, 1, 0)
    with pytest.raises(L.BseError, match="BSE_ERR_WORKSPACE"):
        L.bse_screening(L.BseScreenDesc(**sd), 1, 1, 1, 1, 1, 1, 1, 1, 16, 1, 0)
    assert lib.bse_status_string(2) == b"workspace too small"


def test_coulomb_and_probe_reject_bad_arguments(lib):
    """Argument checks of bse_coulomb and bse_probe, before any device call."""
    import ctypes
    q = (ctypes.c_double * 3)(0.0, 0.0, 0.0)
    for args in ((0, 1, 10.0, q, 1, 1), (5, None, 10.0, q, 1, 1), (5, 1, 0.0, q, 1, 1),
                 (5, 1, float("nan"), q, 1, 1), (5, 1, 10.0, None, 1, 1), (5, 1, 10.0, q, None, 1),
                 (5, 1, 10.0, q, 1, None)):
        assert lib.bse_coulomb(*args, None) == 1
    q[1] = float("inf")
    assert lib.bse_coulomb(5, 1, 10.0, q, 1, 1, None) == 1
    for args in ((0, 5, 1, 1, 1), (4, 0, 1, 1, 1), (4, 5, None, 1, 1), (4, 5, 1, None, 1),
                 (4, 5, 1, 1, None)):
        assert lib.bse_probe(*args, None) == 1


def test_tuning_table_round_trip_and_validation(lib):
    old = L.bse_tune_get()
    try:
        L.bse_tune_set([(0, 4096, 4), (1, 6144, 64), (4, 2000, 16)])
        assert L.bse_tune_get() == [(0, 4096, 4), (1, 6144, 64), (4, 2000, 16)]
        for bad in ([(0, 4096, 3)], [(1, 6144, 48)], [(12, 10, 32)], [(2, 0, 32)], [(6, 100, 10)],
                    [(8, 100, 3)], [(9, 100, 48)], [(10, 100, 2)], [(11, 100, 8)]):
            with pytest.raises(L.BseError, match="BSE_ERR_ARG"):
                L.bse_tune_set(bad)
            assert len(L.bse_tune_get()) == 3  # a rejected table changes nothing
        L.bse_tune_set([])
        assert L.bse_tune_get() == []
    finally:
        L.bse_tune_set(old)

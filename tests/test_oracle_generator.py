"""Pins of the oracle's counter-based generator (the drawn M_{u u'}(G') of
core-level workloads) and of the oracle on workloads that use it.

The generator is pinned by the published known-answer values of Philox4x32-10
and by the distribution of its Box-Muller normals; the assembly with drawn
elements by the literal double sums and by the closed forms that hold for any
pair elements.
"""
import os

import numpy as np
import pytest
from scipy import stats

from bse_synth import get, make_inputs
from bse_synth.generate import mcc_key
from oracle import bse_oracle as O
from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((tuple(v[0:4]), tuple(v[4:6]), tuple(v[6:10])))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    got = tuple(int(x) for x in philox.philox4x32_10(ctr, key))
    assert got == out


def test_philox_vectorised_equals_scalar_calls():
    """Array counters give, element by element, the block of each counter."""
    ctr = (np.arange(5), np.arange(5) * 7, np.full(5, 3), np.arange(5)[::-1])
    key = (0x1234, 0xabcdef)
    arr = philox.philox4x32_10(ctr, key)
    for i in range(5):
        one = philox.philox4x32_10(tuple(int(c[i]) for c in ctr), key)
        assert tuple(int(a[i]) for a in arr) == tuple(int(o) for o in one)


def test_box_muller_normals():
    """z = (x + i y)/sqrt(2) with x, y independent standard normals: KS test of
    x and y against the normal law, E|z|^2 = 1, E z^2 = 0, E|z|^4 = 2."""
    n = 1 << 18
    i = np.arange(n)
    z = philox.complex_normal((i, i >> 7, np.zeros(n, np.int64), np.full(n, 9)), (77, 5))
    x, y = np.sqrt(2.0) * z.real, np.sqrt(2.0) * z.imag
    assert stats.kstest(x, "norm").pvalue > 1e-4
    assert stats.kstest(y, "norm").pvalue > 1e-4
    se = 1.0 / np.sqrt(n)
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 6 * se
    assert abs(np.mean(z * z)) < 6 * se
    assert abs(np.mean(np.abs(z) ** 4) - 2.0) < 6 * 4.5 * se
    assert abs(np.corrcoef(x, y)[0, 1]) < 6 * se


def test_mcc_indexing_and_key():
    """Slices of a pair list equal the draws for those pairs alone; another key
    or another pair gives other values; the envelope multiplies each G."""
    env = np.linspace(1.0, 0.1, 9)
    a = philox.mcc_pairs(mcc_key(get("tiny_core_k2_c2c6_g27")), env, np.arange(6), 3)
    b = philox.mcc_pairs(mcc_key(get("tiny_core_k2_c2c6_g27")), env, [4, 1], 3)
    assert np.array_equal(a[[4, 1]], b)
    c = philox.mcc_pairs(mcc_key(get("mid_core_k4_c2c8_g59")), env, [4, 1], 3)
    assert np.abs(c - b).min() > 0.0
    assert np.abs(a[0] - a[1]).min() > 0.0
    d = philox.mcc_pairs(mcc_key(get("tiny_core_k2_c2c6_g27")), np.ones(9), [4, 1], 3)
    assert np.allclose(b, d * env[None, None, None, :], rtol=0, atol=1e-15)


def test_core_assembly_literal_double_sums():
    """Drawn Mcc: the factorised contraction equals the literal double sums."""
    d = make_inputs(get("tiny_core_k2_c2c6_g27"))
    A, _ = O.assemble(d)
    A2, _ = O.assemble(d, literal=True)
    assert np.abs(A - A2).max() / np.abs(A).max() < 1e-13


def test_core_structure_closed_forms():
    """Flat core levels: the transition energies are eps_c + 400; with the
    kernel off the eigenvalues are those energies; the TDA trace holds; the
    sampled-block route equals the full assembly on drawn elements."""
    d = make_inputs(get("mid_core_k4_c2c8_g59"))
    w = d["workload"]
    E0 = O.transition_energies(d)
    assert np.allclose(E0.reshape(w.nk, w.nv, w.nc), d["eps_c"][:, None, :] + 400.0, atol=1e-12)
    A, _ = O.assemble(d)
    E, _ = O.solve_tda(A)
    assert abs(E.sum() - np.trace(A).real) < 1e-9 * np.abs(E).sum()
    A0, _ = O.assemble(d, bse_type="ip")
    E0s, _ = O.solve_tda(A0)
    assert np.allclose(E0s, np.sort(E0), rtol=0, atol=1e-10)
    ik, jk = O.pairs(w.nk)
    sel = np.array([0, 5, 17, len(ik) - 1])
    blk, _ = O.kernel_blocks(d, sel)
    nvnc = w.nv * w.nc
    for s, b in zip(sel, blk):
        ref = A[ik[s] * nvnc:(ik[s] + 1) * nvnc, jk[s] * nvnc:(jk[s] + 1) * nvnc]
        if ik[s] == jk[s]:
            b = O.hermitian_rule(b)
        assert np.abs(b - ref).max() < 1e-12 * np.abs(A).max()

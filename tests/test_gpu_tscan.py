"""The temperature scan of Sec. 3 (Figs. 3-5) on the batched engine, at a
reduced size: qualitative properties the paper reports and the mapping to
lattice units fixes.  Statistical checks allow five block-average errors."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def scan():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1610_02733_amd import tscan
    rows = tscan.temperature_scan(variants=(1, 2, 3), ns=(1, 10), dts=(0.01,), zetas=(1.0, 20.0),
                                  box=12, n_chains=4, chain_len=64, t_tau=40.0, equil_tau=5.0,
                                  sample_tau=0.5, seed=3)
    for r in rows:
        print(r)
    return {(r["variant"], r["n"], r["zeta"]): r for r in rows}


def _T(scan, variant, n, zeta):
    r = scan[(variant, n, zeta)]
    assert r["finite"], r
    return r["T_over_kT"], r["err"]


def test_small_friction_keeps_temperature(scan):
    for variant in (1, 2, 3):
        T, e = _T(scan, variant, 1, 1.0)
        assert abs(T - 1.0) < max(5 * e, 0.03), (variant, T, e)


def test_variant_a_heats_with_contrast_and_friction(scan):
    """Variant A sees a fluid velocity that is frozen for n MD steps: its
    heating grows with n at large friction (Fig. 3)."""
    Ta1, ea1 = _T(scan, 1, 1, 20.0)
    Ta10, ea10 = _T(scan, 1, 10, 20.0)
    assert Ta10 - Ta1 > 5 * np.hypot(ea1, ea10)
    Tlow, elow = _T(scan, 1, 10, 1.0)
    assert Ta10 - Tlow > 5 * np.hypot(ea10, elow)


def test_variant_b_beats_a_at_large_contrast(scan):
    """At n = 10 and large friction variant B stays much closer to kT than
    variant A (Fig. 4), and variant C is indistinguishable from B (Fig. 5)."""
    Ta, ea = _T(scan, 1, 10, 20.0)
    Tb, eb = _T(scan, 2, 10, 20.0)
    Tc, ec = _T(scan, 3, 10, 20.0)
    assert (Ta - 1.0) - (Tb - 1.0) > 5 * np.hypot(ea, eb)
    assert abs(Tb - Tc) < 5 * np.hypot(eb, ec)


def test_variants_coincide_statistically_at_n1(scan):
    """For n = 1 the three variants are the same algorithm (Sec. 3)."""
    for zeta in (1.0, 20.0):
        T1, e1 = _T(scan, 1, 1, zeta)
        for v in (2, 3):
            T, e = _T(scan, v, 1, zeta)
            assert abs(T - T1) < 5 * np.hypot(e, e1) + 1e-6, (zeta, v, T, T1)

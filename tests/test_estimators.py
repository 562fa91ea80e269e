"""Host estimators of the product package (paper_2103_10449_amd.estimators)
against closed forms and against the oracle's own estimators."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2103_10449_amd import estimators as est

KB = 8.617333262e-5


def test_delta_f_and_heat_match_oracle():
    g = np.random.default_rng(3)
    wf, wb = g.normal(1.0, 0.1, 50), g.normal(-0.7, 0.1, 40)
    assert est.delta_f(wf, wb) == pytest.approx(orc.delta_f(wf, wb), abs=0, rel=1e-15)
    assert est.dissipated_heat(wf, wb) == pytest.approx(orc.q_diss(wf, wb), rel=1e-15)
    assert est.einstein_free_energy_difference(2.0, 7.0, 300.0, 64) == pytest.approx(
        orc.einstein_free_energy_difference(2.0, 7.0, 300.0, 64), rel=1e-15)


def _rs_harmonic_paths(n_atoms, T0, lam_f, n):
    """Quasi-static reversible-scaling work of a classical harmonic crystal:
    with H = lambda U at T0, <U> = 3 N kB T0 / (2 lambda), so the work from 1
    to lambda is (3/2) N kB T0 ln(lambda) and the way back returns it."""
    lam_fwd = np.linspace(1.0, lam_f, n)
    w_fwd = 1.5 * n_atoms * KB * T0 * np.log(lam_fwd)
    lam_bwd = lam_fwd[::-1]
    w_bwd = 1.5 * n_atoms * KB * T0 * (np.log(lam_bwd) - np.log(lam_f))
    return lam_fwd, w_fwd, lam_bwd, w_bwd


def test_gibbs_rs_reproduces_harmonic_free_energy():
    """A classical harmonic crystal has F(T) = 3 N kB T ln(c / T); reversible
    scaling from F(T0) must give F(T0/lambda) for every lambda (eq. Gibbs_RS).
    Dropping the kinetic (3/2) N kB T0 ln(lambda) term or the 1/lambda of the
    work term misses it by O(N kB T0)."""
    N, T0, c = 64, 600.0, 5.0e4
    F = lambda T: 3 * N * KB * T * np.log(c / T)
    lf, wf, lb, wb = _rs_harmonic_paths(N, T0, 2.5, 4001)
    grid = np.linspace(1.0, 2.5, 13)
    T, G = est.gibbs_rs(F(T0), N, T0, lf, wf, lb, wb, grid)
    np.testing.assert_allclose(T, T0 / grid, rtol=1e-15)
    np.testing.assert_allclose(G, F(T), rtol=0, atol=2e-6)
    # each grid point agrees with the oracle's single-lambda formula
    for lam, g in zip(grid, G):
        wfl = 1.5 * N * KB * T0 * np.log(lam)
        assert g == pytest.approx(orc.gibbs_rs(F(T0), lam, N, T0, wfl, -wfl), abs=2e-6)


def test_gibbs_rs_uses_the_backward_work_from_lambda_to_one():
    """Irreversible paths: W(1->lambda) of the forward run and W(lambda->1) =
    W_b(total) - W_b(up to lambda) of the backward run."""
    N, T0 = 10, 300.0
    lf = np.linspace(1.0, 2.0, 101)
    wf = 0.3 * (lf - 1.0) + 0.05 * (lf - 1.0) ** 2
    lb = lf[::-1]
    wb = -0.2 * (2.0 - lb) + 0.01 * (2.0 - lb) ** 3
    lam = 1.6
    _, G = est.gibbs_rs(-1.0, N, T0, lf, wf, lb, wb, [lam])
    w_f = 0.3 * 0.6 + 0.05 * 0.36
    w_b_to_lam = -0.2 * 0.4 + 0.01 * 0.064
    w_b_total = -0.2 + 0.01
    expect = orc.gibbs_rs(-1.0, lam, N, T0, w_f, w_b_total - w_b_to_lam)
    assert G[0] == pytest.approx(expect, abs=5e-6)


def test_gibbs_as_reproduces_ideal_gas():
    """Quasi-static pressure switching of an ideal gas: W = int V dP with
    V = N kB T / P, so G(P) - G(P0) = N kB T ln(P / P0) (eq. Gibbs_AS)."""
    N, T, P0, P1 = 100, 800.0, 0.01, 0.05
    pf = np.linspace(P0, P1, 20001)
    wf = N * KB * T * np.log(pf / P0)
    pb = pf[::-1]
    wb = N * KB * T * np.log(pb / P1)
    grid = np.linspace(P0, P1, 9)
    P, G = est.gibbs_as(-3.0, pf, wf, pb, wb, grid)
    np.testing.assert_allclose(P, grid)
    np.testing.assert_allclose(G, -3.0 + N * KB * T * np.log(grid / P0), atol=1e-9)


def test_dcci_coexistence_scaling():
    T, P = est.dcci_coexistence(1000.0, [1.0, 2.0, 0.5], [3.0, 3.0, 1.0])
    np.testing.assert_allclose(T, [1000.0, 500.0, 2000.0])
    np.testing.assert_allclose(P, [3.0, 1.5, 2.0])


def _constrained_integrals_1d(n, a, b, h=2e-3, L=8.0):
    """Brute-force quadrature of the centre-of-mass-constrained integrals of
    n 1D oscillators: int du delta(sum u / n) exp(-a sum u^2) and
    int dp delta(sum p) exp(-b sum p^2), by eliminating the last coordinate
    on a grid (n = 2: 1D grid, n = 3: 2D grid)."""
    su = np.arange(-L, L + h / 2, h) / np.sqrt(a)
    sp = np.arange(-L, L + h / 2, h) / np.sqrt(b)
    if n == 2:
        zu = n * np.trapezoid(np.exp(-a * (su ** 2 + su ** 2)), su)
        zp = np.trapezoid(np.exp(-b * (sp ** 2 + sp ** 2)), sp)
    else:
        U1, U2 = np.meshgrid(su[::8], su[::8], indexing="ij")
        zu = n * np.trapezoid(np.trapezoid(np.exp(-a * (U1 ** 2 + U2 ** 2 + (U1 + U2) ** 2)), su[::8]), su[::8])
        P1, P2 = np.meshgrid(sp[::8], sp[::8], indexing="ij")
        zp = np.trapezoid(np.trapezoid(np.exp(-b * (P1 ** 2 + P2 ** 2 + (P1 + P2) ** 2)), sp[::8]), sp[::8])
    return zu, zp


@pytest.mark.parametrize("n", [2, 3])
def test_einstein_reference_with_fixed_centre_of_mass_brute_force(n):
    """The absolute Einstein reference (Einstein free energy plus the
    centre-of-mass term) equals -kT ln of the free crystal's integral built
    from brute-force quadratures of the constrained ones: (V / N) (2 pi N m
    kT)^(3/2) Z_pos Z_mom / h^(3N), Z_pos and Z_mom the cubes of the 1D
    constrained position and momentum integrals.  A wrong oscillator count
    (3N instead of 3(N - 1)) or a dropped N^(3/2) fails by kT ln N or more."""
    k, T, mass, V = 6.0, 500.0, 28.0855, 173.0
    kT = KB * T
    m = mass * est.AMU_A2_PS2                  # eV ps^2 / A^2
    zu, zp = _constrained_integrals_1d(n, k / (2 * kT), 1 / (2 * m * kT))
    h = 2 * np.pi * est.HBAR
    lnZ = np.log(V / n) + 1.5 * np.log(2 * np.pi * n * m * kT) + 3 * np.log(zu) + 3 * np.log(zp) - 3 * n * np.log(h)
    F = est.einstein_free_energy(n, k, T, mass) + est.com_correction(n, k, T, V)
    assert F == pytest.approx(-kT * lnZ, abs=1e-9)
    # and the closed forms of the two constrained integrals
    assert zu == pytest.approx(np.sqrt(n) * (np.pi / (k / (2 * kT))) ** ((n - 1) / 2), rel=1e-9)
    assert zp == pytest.approx((np.pi * 2 * m * kT) ** ((n - 1) / 2) / np.sqrt(n), rel=1e-9)


def test_solid_free_energy_and_coexistence_pressure():
    """F = Einstein reference - dF(crystal -> Einstein); two phases with
    linear g(P) cross where the first-order estimate says."""
    N, k, T, m, V = 512, 7.0, 400.0, 28.0855, 512 * 20.0
    ref = est.einstein_free_energy(N, k, T, m) + est.com_correction(N, k, T, V)
    wf, wb = np.array([3.0, 3.2]), np.array([-2.0, -2.2])
    assert est.solid_free_energy(N, k, T, m, V, wf, wb) == pytest.approx(ref - 0.5 * (3.1 + 2.1))
    g1, v1, g2, v2, P = -4.30, 19.0, -4.31, 16.0, 13.0
    Pc = est.coexistence_pressure(P, g1, v1, g2, v2)
    c = est.EV_A3_PER_GPA
    assert g1 + v1 * (Pc - P) * c == pytest.approx(g2 + v2 * (Pc - P) * c, abs=1e-14)
    assert Pc < P  # the denser phase 2 is lower in g at P, so the crossing is below P


def test_ideal_gas_entropy_is_sackur_tetrode_argon():
    """S = -dF/dT of the ideal gas at fixed V for argon (39.948 amu) at
    298.15 K and 1 bar: the tabulated standard molar entropy, 154.8 J/(mol
    K), pins the thermal wavelength (hbar, the amu conversion, kB)."""
    T, P_bar, m = 298.15, 1.0, 39.948
    N = 10 ** 6
    V = N * KB * T / (P_bar * 1e5 / 1.602176634e-19 * 1e-30)   # A^3
    h = 1e-3
    S = -(est.ideal_gas_free_energy(N, V, T + h, m) - est.ideal_gas_free_energy(N, V, T - h, m)) / (2 * h)
    S_molar = S / N * 1.602176634e-19 * 6.02214076e23                 # J/(mol K)
    assert S_molar == pytest.approx(154.8, abs=0.1)


def test_transition_temperature_and_liquid_assembly():
    """Phases with g_i(T') = h_i + (g_i(T) - h_i) T'/T (constant h, linear
    entropy term) cross where the first-order estimate says; the liquid
    assembly adds the two switching free energies with the right signs."""
    T, g1, h1, g2, h2 = 1600.0, -4.10, -3.90, -4.08, -3.50
    Tt = est.transition_temperature(T, g1, h1, g2, h2)
    g = lambda gi, hi: hi + (gi - hi) * Tt / T
    assert g(g1, h1) == pytest.approx(g(g2, h2), abs=1e-12)
    F = est.liquid_free_energy(100, 2000.0, T, 28.0855, [1.0], [-0.8], [-3.0], [3.4])
    assert F == pytest.approx(est.ideal_gas_free_energy(100, 2000.0, T, 28.0855) + 0.9 - (-3.2))


def test_gibbs_estimators_with_logs_that_skip_the_start():
    """Logs read from the library hold their first row one logging interval
    after the schedule start, not the start itself.  Given the schedule starts,
    the estimators anchor W = 0 there: the ideal-gas G(P) and the harmonic
    G(T) come out as from logs that hold the start, while anchoring at the
    first logged row would be off by the work of one interval."""
    N, T, P0, P1, n, every = 100, 800.0, 0.01, 0.05, 20000, 500
    pf = np.linspace(P0, P1, n + 1)
    wf = N * KB * T * np.log(pf / P0)
    pb = pf[::-1]
    wb = N * KB * T * np.log(pb / P1)
    grid = np.linspace(P0, P1, 9)
    rows = slice(every, None, every)          # rows after every `every` steps
    _, G = est.gibbs_as(-3.0, pf[rows], wf[rows], pb[rows], wb[rows], grid, p0=P0, p1=P1)
    exact = -3.0 + N * KB * T * np.log(grid / P0)
    np.testing.assert_allclose(G, exact, atol=2e-3)
    _, G_bad = est.gibbs_as(-3.0, pf[rows], wf[rows], pb[rows], wb[rows], grid)
    assert np.abs(G_bad - exact).max() > 10 * np.abs(G - exact).max()

    N, T0, c, lam_f = 64, 600.0, 5.0e4, 2.5
    F = lambda T: 3 * N * KB * T * np.log(c / T)
    lf, wfl, lb, wbl = _rs_harmonic_paths(N, T0, lam_f, 4001)
    rows = slice(100, None, 100)
    lam_grid = np.linspace(1.0, lam_f, 13)
    T, G = est.gibbs_rs(F(T0), N, T0, lf[rows], wfl[rows], lb[rows], wbl[rows], lam_grid, lam_f=lam_f)
    np.testing.assert_allclose(G, F(T), atol=2e-3)

"""Pins for the oracle's Stillinger-Weber energy, forces, virial and gradients.

Everything here checks the oracle against facts fixed independently of its
own code: lattice sums with hand-derived angular coefficients, the published
normalisation of the 1985 silicon parameters, periodic-replication
invariance, finite differences, symmetry and exact scaling identities.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2103_10449_amd import inputs

R6 = 2.0 ** (1.0 / 6.0)


def _g(r, P):
    return np.exp(P["gamma"] * P["sigma"] / (r - P["a"] * P["sigma"]))


def test_diamond_cohesive_energy_is_minus_two_epsilon(sw_params):
    """The 1985 parameters put the pair minimum at r = 2^(1/6) sigma with depth
    -epsilon; at the matching lattice constant a0 = 4 * 2^(1/6) sigma / sqrt(3)
    each diamond atom has 4 neighbours at tetrahedral angles, so E/N = -2 eps
    and the three-body sum vanishes exactly."""
    P = sw_params
    a0 = 4.0 * R6 * P["sigma"] / np.sqrt(3.0)
    x, box = inputs.diamond((3, 3, 3), a0)
    r = orc.sw_eval(x, box, P)
    n = len(x)
    assert r["E3"] == pytest.approx(0.0, abs=1e-12 * n)
    assert r["E"] / n == pytest.approx(-2.0 * P["epsilon"], rel=1e-8)
    # pair minimum: zero stress at a0
    assert np.abs(r["virial"]).max() < 1e-7 * n
    assert np.all(r["nnb"] == 4)
    # and at the paper-era lattice constant 5.431 A the value is the familiar -4.3366 eV
    x, box = inputs.diamond((2, 2, 2), 5.431)
    r = orc.sw_eval(x, box, P)
    assert r["E"] / len(x) == pytest.approx(-4.3366, abs=2e-4)


@pytest.mark.parametrize("a_sc", [2.7, 2.9, 3.3])
def test_three_body_lattice_sums_sc_fcc(sw_params, a_sc):
    """Hand-derived angular sums.  Simple cubic with 6 neighbours at distance d:
    12 pairs at 90 deg, 3 at 180 deg -> sum (cos - c0)^2 = 12/9 + 3*(4/9) = 8/3.
    fcc with 12 neighbours at d: 24 at 60, 12 at 90, 24 at 120, 6 at 180 deg
    -> 24*(25/36) + 12*(4/36) + 24*(1/36) + 6*(16/36) = 64/3.
    So E3/N = lam*eps*g(d)^2 * {8/3, 64/3}, E2/N = {3, 6} * phi2(d)."""
    P = sw_params
    d = a_sc
    if np.sqrt(2.0) * d < P["a"] * P["sigma"]:
        pytest.skip("second shell inside the cutoff")
    xs, bs = inputs.simple_cubic((4, 4, 4), d)
    xf, bf = inputs.fcc((3, 3, 3), d * np.sqrt(2.0))
    rs, rf = orc.sw_eval(xs, bs, P), orc.sw_eval(xf, bf, P)
    le = P["lambda_sw"] * P["epsilon"]
    g2 = _g(d, P) ** 2
    assert rs["E3"] / len(xs) == pytest.approx(le * g2 * 8.0 / 3.0, rel=1e-12)
    assert rf["E3"] / len(xf) == pytest.approx(le * g2 * 64.0 / 3.0, rel=1e-12)
    # pair sums scale with the coordination number only
    assert (rf["E2"] / len(xf)) / (rs["E2"] / len(xs)) == pytest.approx(2.0, rel=1e-12)
    assert np.all(rs["nnb"] == 6) and np.all(rf["nnb"] == 12)


def test_explicit_images_equal_supercell(sw_params):
    """An 8-atom diamond cell (L < 2 r_c, explicit image sum) and its 2x2x2
    replica (minimum image) describe the same periodic crystal: energy per
    atom, per-atom energies and forces must agree."""
    P = sw_params
    g = inputs.rng(900, 0, 0)
    x1, b1 = inputs.diamond((1, 1, 1), 5.431)
    x1 = x1 + g.normal(0, 0.08, size=x1.shape)
    shifts = np.array([[i, j, k] for i in range(2) for j in range(2) for k in range(2)], float)
    x8 = (x1[None, :, :] + shifts[:, None, :] * b1[None, None, :]).reshape(-1, 3)
    r1 = orc.sw_eval(x1, b1, P)
    r8 = orc.sw_eval(x8, 2 * b1, P)
    assert r8["E"] == pytest.approx(8 * r1["E"], rel=1e-12)
    assert np.allclose(r8["F"].reshape(8, 8, 3), r1["F"][None], atol=1e-11)
    assert np.allclose(r8["virial"], 8 * r1["virial"], atol=1e-10)


def test_minimum_image_equals_explicit_images(sw_params):
    P = sw_params
    x, box = inputs.random_box(40, 9.0, inputs.rng(901, 0, 0))
    a = orc.sw_eval(x, box, P, force_images=False)
    b = orc.sw_eval(x, box, P, force_images=True)
    assert a["E"] == pytest.approx(b["E"], rel=1e-13)
    assert np.allclose(a["F"], b["F"], atol=1e-12)


def _rand_cfg(seed, n=48, L=9.5):
    return inputs.random_box(n, L, inputs.rng(902, seed, 0), d_min=2.05)


@pytest.mark.parametrize("seed", [0, 1])
def test_forces_finite_difference(sw_params, seed):
    P = sw_params
    x, box = _rand_cfg(seed)
    r = orc.sw_eval(x, box, P)
    h = 1e-5
    g = inputs.rng(903, seed, 0)
    fmax = max(np.abs(r["F"]).max(), 1.0)
    for i in g.choice(len(x), 8, replace=False):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = -(orc.sw_eval(xp, box, P)["E"] - orc.sw_eval(xm, box, P)["E"]) / (2 * h)
            assert abs(fd - r["F"][i, a]) < 1e-7 * fmax


def test_net_force_zero_and_virial_symmetric(sw_params):
    P = sw_params
    x, box = _rand_cfg(3, n=64, L=10.5)
    r = orc.sw_eval(x, box, P)
    fs = np.abs(r["F"]).max()
    assert np.abs(r["F"].sum(axis=0)).max() < 1e-12 * fs * len(x)
    assert np.allclose(r["virial"], r["virial"].T, atol=1e-10 * np.abs(r["virial"]).max())


def test_virial_finite_difference_including_shear(sw_params):
    """Xi_ab = dE/d strain_ab with r -> (I + strain) r and the cell deformed with it."""
    P = sw_params
    x, box = _rand_cfg(4)
    r = orc.sw_eval(x, box, P)
    h = 1e-5
    H0 = np.diag(box)
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = h
            Ep = orc.sw_eval(x @ (np.eye(3) + e).T, (np.eye(3) + e) @ H0, P)["E"]
            Em = orc.sw_eval(x @ (np.eye(3) - e).T, (np.eye(3) - e) @ H0, P)["E"]
            fd = (Ep - Em) / (2 * h)
            assert fd == pytest.approx(r["virial"][a, b], abs=2e-7 * max(1.0, np.abs(r["virial"]).max()))


def test_parameter_gradient_identities(sw_params):
    """Exact identities: dE/deps = E/eps, dE/dA = E2/A, dE/dlam = E3/lam, and the
    scale invariance of SW in r/sigma: sigma dE/dsigma = -tr(Xi)."""
    P = sw_params
    x, box = _rand_cfg(5)
    r = orc.sw_eval(x, box, P)
    G = dict(zip(orc.PARAM_NAMES, r["dtheta"]))
    assert G["epsilon"] == pytest.approx(r["E"] / P["epsilon"], rel=1e-12)
    assert G["A"] == pytest.approx(r["E2"] / P["A"], rel=1e-12)
    assert G["lambda_sw"] == pytest.approx(r["E3"] / P["lambda_sw"], rel=1e-12)
    assert P["sigma"] * G["sigma"] == pytest.approx(-np.trace(r["virial"]), rel=1e-9)


@pytest.mark.parametrize("name", ["B", "p", "q", "a", "gamma", "sigma"])
def test_parameter_gradient_finite_difference(sw_params, name):
    P = sw_params
    x, box = _rand_cfg(6)
    r = orc.sw_eval(x, box, P)
    key = name
    i = orc.PARAM_NAMES.index(key)
    h = 1e-5 * max(1.0, abs(P[key]))
    Pp, Pm = dict(P), dict(P)
    Pp[key] += h
    Pm[key] -= h
    fd = (orc.sw_eval(x, box, Pp)["E"] - orc.sw_eval(x, box, Pm)["E"]) / (2 * h)
    assert fd == pytest.approx(r["dtheta"][i], rel=1e-6, abs=1e-6)


def test_symmetries(sw_params):
    """Translation, atom relabelling and axis permutation leave E unchanged."""
    P = sw_params
    x, box = _rand_cfg(7, n=40, L=9.8)
    box = np.array([9.8, 10.3, 11.1])
    x = x * box / 9.8
    E = orc.sw_eval(x, box, P)["E"]
    assert orc.sw_eval(x + np.array([1.3, -7.1, 22.0]), box, P)["E"] == pytest.approx(E, rel=1e-12)
    perm = inputs.rng(904, 0, 0).permutation(len(x))
    assert orc.sw_eval(x[perm], box, P)["E"] == pytest.approx(E, rel=1e-12)
    assert orc.sw_eval(x[:, [2, 0, 1]], box[[2, 0, 1]], P)["E"] == pytest.approx(E, rel=1e-12)


def test_beta_sn_neighbour_count(sw_params):
    """beta-tin at a = 4.80, c = 2.65: 4 neighbours at 2.49, 2 at 2.65, 4 at 3.12
    and 8 at 3.64 A all lie inside r_c = 3.77 A, so every atom has 18."""
    x, box = inputs.beta_sn((4, 4, 8), 4.80, 2.65)
    r = orc.sw_eval(x, box, sw_params)
    assert np.all(r["nnb"] == 18)


def test_einstein_reference():
    g = inputs.rng(905, 0, 0)
    x0 = g.normal(size=(10, 3))
    x = x0 + g.normal(scale=0.1, size=x0.shape)
    U, F = orc.einstein(x, x0, 3.0)
    assert U == pytest.approx(0.5 * 3.0 * ((x - x0) ** 2).sum(), rel=1e-14)
    h = 1e-6
    xp = x.copy()
    xp[2, 1] += h
    xm = x.copy()
    xm[2, 1] -= h
    fd = -(orc.einstein(xp, x0, 3.0)[0] - orc.einstein(xm, x0, 3.0)[0]) / (2 * h)
    assert fd == pytest.approx(F[2, 1], rel=1e-8)


# ------------------------------------------------ Uhlenbeck-Ford reference ----
UF = dict(p=25.0, sigma=2.0, T=2200.0)


def test_uf_second_virial_coefficient_closed_form():
    """The oracle's UF pair energy, through its Mayer function
    f(r) = exp(-phi(r)/kB T) - 1 = (1 - exp(-(r/s)^2))^p - 1 at the model's
    own temperature, integrates to the closed form
    B2 = -2 pi int f r^2 dr = (pi^(3/2) s^3 / 2) sum_k (-1)^(k+1) C(p,k) k^(-3/2)
    (binomial expansion and Gaussian integrals); 129.86 A^3 for p = 25,
    s = 2 A.  A wrong exponent, p, sigma or temperature scaling fails this."""
    from math import comb, fsum, pi
    from scipy.integrate import quad
    p, s, T = UF["p"], UF["sigma"], UF["T"]
    rcut = 12 * s
    box = np.array([4 * rcut] * 3)

    def f(r):
        x = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
        e = orc.uf_eval(x, box, p, s, T, rcut)["E"]
        return (np.exp(-e / (orc.KB * T)) - 1.0) * r * r

    integral = quad(f, 1e-6, rcut, limit=200, epsabs=1e-12, epsrel=1e-11)[0]
    B2 = -2 * pi * integral
    closed = pi ** 1.5 * s ** 3 / 2 * fsum((-1) ** (k + 1) * comb(int(p), k) * k ** -1.5 for k in range(1, int(p) + 1))
    assert closed == pytest.approx(129.861039, rel=1e-6)
    assert B2 == pytest.approx(closed, rel=1e-8)


def test_uf_forces_and_virial_finite_difference():
    x, box = inputs.liquid_rsa(64, inputs.rng(904, 0, 0))
    r = orc.uf_eval(x, box, UF["p"], UF["sigma"], UF["T"], 8.0)
    fs = max(np.abs(r["F"]).max(), 1.0)
    assert np.abs(r["F"].sum(axis=0)).max() < 1e-11 * fs * len(x)
    h = 1e-5
    g = inputs.rng(904, 0, 1)
    for i in g.choice(len(x), 6, replace=False):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            fd = -(orc.uf_eval(xp, box, UF["p"], UF["sigma"], UF["T"], 8.0)["E"]
                   - orc.uf_eval(xm, box, UF["p"], UF["sigma"], UF["T"], 8.0)["E"]) / (2 * h)
            assert abs(fd - r["F"][i, a]) < 1e-7 * fs
    H0 = np.diag(box)
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = h
            Ep = orc.uf_eval(x @ (np.eye(3) + e).T, (np.eye(3) + e) @ H0, UF["p"], UF["sigma"], UF["T"], 8.0)["E"]
            Em = orc.uf_eval(x @ (np.eye(3) - e).T, (np.eye(3) - e) @ H0, UF["p"], UF["sigma"], UF["T"], 8.0)["E"]
            assert (Ep - Em) / (2 * h) == pytest.approx(r["virial"][a, b], abs=1e-6 * max(1.0, np.abs(r["virial"]).max()))


def test_uf_minimum_image_equals_explicit_images():
    x, box = inputs.liquid_rsa(512, inputs.rng(904, 1, 0))
    assert box.min() > 2 * 7.0
    a = orc.uf_eval(x, box, UF["p"], UF["sigma"], UF["T"], 7.0)
    b = orc.uf_eval(x, box, UF["p"], UF["sigma"], UF["T"], 7.0, force_images=True)
    assert a["E"] == pytest.approx(b["E"], rel=1e-13)
    assert np.allclose(a["F"], b["F"], atol=1e-12)


def test_thread_count_changes_no_result(sw_params):
    """The neighbour search may run on several threads; each atom's list is
    built alone and in the same order, so every output is bitwise the same."""
    x, box = inputs.liquid_rsa(700, inputs.rng(990, 0, 0))
    out = []
    for n in (1, 4):
        orc.set_threads(n)
        out.append(orc.sw_eval(x, box, sw_params))
    orc.set_threads(1)
    a, b = out
    assert a["E2"] == b["E2"] and a["E3"] == b["E3"]
    for k in ("F", "virial", "dtheta", "e_atom", "nnb"):
        assert np.array_equal(a[k], b[k]), k

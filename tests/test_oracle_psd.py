"""Pins of the oracle's PSD estimator (Sec. 3.2, Alg. 2) to closed forms.

Each check is fixed by the mathematics, not by the oracle's own formulas:
quadrature of the ball jump kernel, the sampler's distribution against its
cumulative distribution, tangent-ball radii of a box, the unit ball's
Dirichlet form of textbook spherical harmonics, and the PSD structure.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from paper_2606_05581_amd import workloads as W


def _jump(theta, r):
    """Ball jump kernel 1 / (2 pi |s - z|^3) at polar angle theta about s (eq. ball-jump-kernel)."""
    return 1.0 / (2.0 * math.pi * (2.0 * r * math.sin(0.5 * theta)) ** 3)


@pytest.mark.parametrize("r", [0.3, 1.0, 2.5])
@pytest.mark.parametrize("cap_deg", [2.5, 10.0])
def test_jump_mass_is_the_kernel_integral(oracle_mod, r, cap_deg):
    """Z = integral of J over the ball sphere outside the cap, by quadrature
    in the polar angle (area element 2 pi r^2 sin theta)."""
    t0 = math.radians(cap_deg)
    ref, err = integrate.quad(lambda t: _jump(t, r) * 2.0 * math.pi * r * r * math.sin(t), t0, math.pi,
                              epsabs=0, epsrel=1e-12, limit=200)
    assert oracle_mod.ball_jump_mass(r, t0) == pytest.approx(ref, rel=1e-9)


def test_ball_points_follow_the_jump_kernel(oracle_mod):
    """Ball points lie on the sphere, outside the cap, with |s - z| distributed
    as J times the area element (KS test against the integrated density), a
    uniform azimuth, and antithetic partners mirrored about the axis c -> s."""
    rng = np.random.default_rng(5)
    c = np.array([0.2, -0.1, 0.4])
    n = np.array([1.0, 2.0, -2.0]) / 3.0
    r, t0 = 0.7, math.radians(2.5)
    s = c + r * n
    xi, eta = rng.random(4000), rng.random(4000)
    Z = np.array([oracle_mod.ball_point(c, r, n, t0, a, b) for a, b in zip(xi, eta)])
    Zp = np.array([oracle_mod.ball_point(c, r, n, t0, a, b, 1) for a, b in zip(xi, eta)])
    assert np.allclose(np.linalg.norm(Z - c, axis=1), r, rtol=1e-12)
    theta = np.arccos(np.clip((Z - c) @ n / r, -1, 1))
    assert theta.min() >= t0 * (1 - 1e-9)
    # CDF of theta from the density 2 pi r^2 sin(theta) J(theta) on [t0, pi]
    mass = oracle_mod.ball_jump_mass(r, t0)

    def cdf(t):
        return np.array([integrate.quad(lambda x: _jump(x, r) * 2 * math.pi * r * r * math.sin(x), t0, ti)[0]
                         for ti in np.atleast_1d(t)]) / mass

    ks = stats.kstest(theta, cdf)
    assert ks.pvalue > 1e-3, ks
    # azimuth about the axis: uniform
    e = (Z - c) / r - np.cos(theta)[:, None] * n
    ref = np.cross(n, [0.0, 0.0, 1.0])
    ref /= np.linalg.norm(ref)
    phi = np.arctan2(e @ np.cross(n, ref), e @ ref)
    assert stats.kstest((phi + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-3
    # partners: same polar angle, opposite azimuth
    mid = 0.5 * (Z + Zp)
    assert np.allclose(mid, c + r * np.cos(theta)[:, None] * n, atol=1e-12)
    assert np.linalg.norm(s - Z, axis=1).min() > 2 * r * math.sin(0.5 * t0) * (1 - 1e-9)


def test_tangent_ball_radii_of_a_box(oracle_mod):
    """In the box [-a,a] x [-b,b] x [-c,c] the largest ball tangent at a point
    of the x = a face is limited by the side faces: r = min(a, distance to the
    nearest side face line in the face); the bisection returns it to within
    r_max / 2^10 (r_max = half the shortest side = min(a, b, c))."""
    a, b, c = 0.9, 0.6, 0.75
    V, F = W.box_grid(6, half=(a, b, c))
    sc = oracle_mod.Scene(V.astype(np.float32), F, bvh=True)
    r_max = oracle_mod.psd_r_max(V)
    assert r_max == pytest.approx(min(a, b, c), rel=1e-6)
    nrm = np.array([1.0, 0.0, 0.0])
    cases = [((a, 0.0, 0.0), min(a, b, c)), ((a, b - 0.2, 0.0), 0.2), ((a, 0.1, -c + 0.05), 0.05),
             ((a, b - 0.45, c - 0.3), 0.3)]
    step = r_max / 2 ** 10
    for s, want in cases:
        r = oracle_mod.tangent_ball(sc, np.array(s), nrm, r_max)
        assert want - 2 * step <= r <= want + 1e-12, (s, r, want)


def _sh_l2(P):
    """Real spherical harmonics of degree <= 2, orthonormal on the unit sphere
    (textbook forms), at unit vectors P; columns grouped by degree 0, 1, 1, 1, 2 x 5."""
    x, y, z = P[:, 0], P[:, 1], P[:, 2]
    c0 = 0.5 / math.sqrt(math.pi)
    c1 = math.sqrt(3.0 / (4 * math.pi))
    c2 = math.sqrt(15.0 / (4 * math.pi))
    c20 = math.sqrt(5.0 / (16 * math.pi))
    c22 = math.sqrt(15.0 / (16 * math.pi))
    cols = [np.full_like(x, c0), c1 * y, c1 * z, c1 * x, c2 * x * y, c2 * y * z, c20 * (3 * z * z - 1), c2 * x * z,
            c22 * (x * x - y * y)]
    return np.stack(cols, 1), [0, 1, 1, 1, 2, 2, 2, 2, 2]


def _ball_form(l, t0):
    """Expected diagonal entry for an orthonormal degree-l harmonic on the unit
    ball with the cap of angle t0 left out: by the Funk-Hecke formula the
    Beurling-Deny form (eq. beurling-deny-bilinear with the ball's kernel)
    reduces to 2 pi int J(theta) (1 - P_l(cos theta)) sin theta dtheta."""
    from scipy.special import eval_legendre

    f = lambda t: 2 * math.pi * _jump(t, 1.0) * (1 - eval_legendre(l, math.cos(t))) * math.sin(t)
    return integrate.quad(f, t0, math.pi, epsabs=0, epsrel=1e-11, limit=200)[0]


def test_ball_form_without_cap_is_the_steklov_eigenvalue():
    """Pin of the pin: without the cap the form is the unit ball's Steklov
    eigenvalue l (the DtN map multiplies degree-l harmonics by l)."""
    for l in (1, 2, 3):
        assert _ball_form(l, 1e-7) == pytest.approx(l, abs=1e-5)


@pytest.fixture(scope="module")
def sphere_psd(oracle_mod):
    V, F = W.icosphere_recursive(4)
    V = V / np.linalg.norm(V, axis=1, keepdims=True)
    rng = np.random.default_rng(21)
    rows = W.point_rows(V, F, 1500, rng)
    tab, deg = _sh_l2(V)
    sc = oracle_mod.Scene(V.astype(np.float32), F, bvh=True)
    out = oracle_mod.psd_estimate(sc, rows, tab, pairs=64, eps=1e-4, seed=3, nthreads=8)
    return out, deg


def _capped_form(l, t0, rbar):
    """Expected entry of an orthonormal degree-l harmonic on the unit sphere when
    tangent balls of mean radius rbar leave out caps of angle t0: the cap about
    s spans |s - z| < rho0 = 2 r sin(t0 / 2), the walk from such z ends next to
    z, and to first order in the cap the left-out part is
    1/2 int (1/2 |grad Y|^2 rho0) ds = 1/2 sin(t0 / 2) l (l + 1) rbar
    (int |grad Y|^2 = l (l + 1)). For r = 1 and l = 1 this is exact."""
    return l - 0.5 * math.sin(0.5 * t0) * l * (l + 1) * rbar


def test_capped_form_matches_ball_quadrature():
    """Pin of the pin: at r = 1 the first-order cap term agrees with the exact
    Funk-Hecke quadrature (exactly for l = 1, to O(t0^2) relative for l = 2)."""
    t0 = math.radians(2.5)
    assert _capped_form(1, t0, 1.0) == pytest.approx(_ball_form(1, t0), rel=1e-9)
    assert _capped_form(2, t0, 1.0) == pytest.approx(_ball_form(2, t0), rel=2e-3)


def test_unit_sphere_harmonics_closed_form(oracle_mod, sphere_psd):
    """Alg. 2 on a fine polyhedral unit sphere with degree <= 2 harmonics: the
    diagonal matches the unit ball's Steklov eigenvalue l less the left-out
    caps, and the off-diagonal vanishes, within 4 standard errors plus 3% for
    the polyhedral surface and the interpolated basis. A dropped weight factor
    (|dOmega|/2, the jump-kernel mass, the pair average) or a wrong sampling
    density fails this. Tangent balls on a polyhedron are bounded by the
    edges (r <= 2 delta / alpha at distance delta from an edge of dihedral
    turn alpha), so radii spread over (0, 1]."""
    out, deg = sphere_psd
    S, se = out["S"], out["se"]
    t0 = math.radians(oracle_mod.PSD_CAP_DEG)
    rad = out["radius"]
    assert np.all(rad > 0) and np.all(rad <= 1.0)
    # constants are in the null space (up to the FP32 rounding of the sample barycentrics)
    assert abs(S[0, 0]) < 1e-12 and np.abs(S[0]).max() < 1e-7 * np.abs(S).max()
    rbar = float(np.mean(rad))
    E = {l: _capped_form(l, t0, rbar) for l in (1, 2)}
    for i in range(1, S.shape[0]):
        want = E[deg[i]]
        assert abs(S[i, i] - want) <= 4 * se[i, i] + 0.03 * want, (i, S[i, i], want, se[i, i])
        for j in range(1, S.shape[0]):
            if j != i:
                assert abs(S[i, j]) <= 4 * se[i, j] + 0.03 * E[2], (i, j, S[i, j])


def test_psd_symmetric_and_positive_on_a_nonconvex_soup(oracle_mod):
    """Every update is alpha d d^T with alpha >= 0, so the estimate is symmetric
    positive semidefinite whatever the geometry (Sec. 3.2, Guaranteeing a PSD
    estimate): a torus soup with a coordinate / quadratic basis."""
    V, F = W.torus_grid(24, 12, 0.6, 0.25, weld_seam=False)
    rng = np.random.default_rng(8)
    rows = W.point_rows(V, F, 300, rng)
    P = V.astype(np.float64)
    tab = np.stack([np.ones(len(P)), P[:, 0], P[:, 1], P[:, 2], P[:, 0] * P[:, 1], P[:, 2] ** 2 - P[:, 0] ** 2], 1)
    sc = oracle_mod.Scene(V.astype(np.float32), F, bvh=True)
    out = oracle_mod.psd_estimate(sc, rows, tab, pairs=16, eps=1e-3, seed=4, nthreads=8, log=True)
    S = out["S"]
    assert np.array_equal(S, S.T) or np.abs(S - S.T).max() <= 1e-15 * np.abs(S).max()
    lam = np.linalg.eigvalsh(0.5 * (S + S.T))
    assert lam.min() >= -1e-12 * lam.max()
    assert np.abs(S[0]).max() < 1e-7 * np.abs(S).max()  # constant column: FP32 barycentric rounding only
    assert np.all(out["radius"] > 0) and np.all(out["radius"] <= 0.25 + 1e-9)
    assert np.all(out["log_status"] != oracle_mod.ESCAPED)

"""Pins for the reverse-Grangeat oracle (oracle.grangeat, Section 2.2.2,
eq 2.21-2.24): Grangeat's relation on a Gaussian (de-postweighting and
pre-weighting against quadrature of closed-form cone-beam projections), the
2D inversion from derivative data on a 2D Gaussian, the 2D NUFFT transpose
against the exact sum, the whole step against closed-form cone-beam line
integrals, and planted mistakes."""
import math

import numpy as np
import pytest

from oracle import grangeat, umbrella

C0 = np.array([1.0, -0.5, 0.8])
COV = np.diag([2.5, 3.0, 2.2]) ** 2
# off the axis, where the pre- and post-weights differ from 1 by ~1 %; its
# shadow stays inside the detector's inscribed disc, as the 2D Radon
# inversion needs (the umbrella lines reach |s| <= side/2 only)
C_OFF = np.array([0.0, 7.0, -6.0])
COV_OFF = np.diag([1.4, 1.5, 1.3]) ** 2
# tap sets switch asymmetrically where a polar frequency's grid coordinate
# ties (the neighbour rule); the imaginary part it leaves is of the order of
# the KB kernel's edge value (~1e-4 at J = 5), far below this
IMAG = 1e-5


def _dradon(rho, n, c, cov):
    s2 = n @ cov @ n
    mass = (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(cov))
    R = mass * np.exp(-(rho - n @ c) ** 2 / (2 * s2)) / math.sqrt(2 * math.pi * s2)
    return -(rho - n @ c) / s2 * R


def _ray(src, p, c, cov):
    """Line integral of exp(-x^T cov^-1 x / 2) (centred at c) along the ray src -> p."""
    A = np.linalg.inv(cov)
    r = (p - src) / np.linalg.norm(p - src)
    d = src - c
    a, b, e = r @ A @ r, r @ A @ d, d @ A @ d
    return math.sqrt(2 * math.pi / a) * math.exp(-0.5 * (e - b * b / a))


def _frame(sc, k, n_proj):
    lam = 2 * math.pi * k / n_proj
    shat = np.array([math.cos(lam), math.sin(lam), 0.0])
    src = sc.R * shat
    return src, src - sc.D * shat, np.array([-math.sin(lam), math.cos(lam), 0.0]), np.array([0.0, 0.0, 1.0])


def _closed_projection(sc, k, n_proj, c=C0, cov=COV):
    src, cdet, uu, vv = _frame(sc, k, n_proj)
    n = sc.n
    X = np.empty((n, n))
    for b in range(n):
        for a in range(n):
            X[b, a] = _ray(src, cdet + (a - n // 2) * sc.delta * uu + (b - n // 2) * sc.delta * vv, c, cov)
    return X


def _umbrella_values(sc, n_proj, c=C0, cov=COV):
    nh, rho = umbrella.geometry(sc.N, n_proj, sc.n_alpha, sc.n)
    return np.array([_dradon(r, v, c, cov) for r, v in zip(rho, nh)]).reshape(n_proj, sc.n_alpha, sc.n)


def test_grangeat_relation_on_a_gaussian():
    # dS/ds' of the pre-weighted projection's 2D Radon transform on the virtual
    # detector, by quadrature of closed-form line integrals and central
    # differences, equals the de-postweighted umbrella value
    sc = grangeat.Scan(32, 16, 32)
    n_proj, k = 3, 1
    U = _umbrella_values(sc, n_proj)[k]
    p = grangeat.depostweight(U, sc).real
    src, cdet, uu, vv = _frame(sc, k, n_proj)

    def g(uv, vv_):  # pre-weighted projection at virtual-detector coordinates
        up, vp = uv, vv_
        X = _ray(src, cdet + (up * sc.D / sc.R) * uu + (vp * sc.D / sc.R) * vv, C0, COV)
        return X * sc.R / math.sqrt(sc.R ** 2 + up ** 2 + vp ** 2)

    tau = np.linspace(-40.0, 40.0, 4001)

    def S(al, s):
        pts = [g(s * math.cos(al) - t * math.sin(al), s * math.sin(al) + t * math.cos(al)) for t in tau]
        return np.trapezoid(pts, tau)

    h = 1e-3
    for i, j in [(0, 14), (3, 17), (5, 12), (9, 18), (13, 15)]:
        al, s = sc.alpha[i], sc.s_v[j]
        dS = (S(al, s + h) - S(al, s - h)) / (2 * h)
        assert abs(dS - p[i, j]) < 1e-5 * np.max(np.abs(p)), (i, j, dS, p[i, j])


@pytest.mark.parametrize("c2,B", [((0.8, -0.6), ((4.0, 1.0), (1.0, 3.0))),
                                  ((6.0, -5.0), ((2.0, 0.5), (0.5, 1.6)))])
def test_2d_inversion_from_derivative_data(c2, B):
    # steps 2-3 alone on a 2D Gaussian image g(u', v'): its derivative 2D Radon
    # transform in closed form -> radial spectra -> NUFFT transpose -> g
    sc = grangeat.Scan(32, 96, 48)
    c2 = np.array(c2)
    B = np.array(B)
    th = np.stack([np.cos(sc.alpha), np.sin(sc.alpha)], 1)
    s = sc.s_v
    sig2 = np.einsum("ia,ab,ib->i", th, B, th)[:, None]
    mu = (th @ c2)[:, None]
    mass = 2 * math.pi * math.sqrt(np.linalg.det(B))
    Sx = mass * np.exp(-(s[None, :] - mu) ** 2 / (2 * sig2)) / np.sqrt(2 * math.pi * sig2)
    dS = -(s[None, :] - mu) / sig2 * Sx
    c = grangeat.radial_spectra(dS, sc)
    g = grangeat.nufft2_adjoint(c, grangeat.polar_omega(sc), sc.n, sc.J, sc.beta)
    U_, V_ = np.meshgrid(s, s)   # [b][a] = (v, u)
    X = np.stack([U_ - c2[0], V_ - c2[1]], -1)
    want = np.exp(-0.5 * np.einsum("bai,ij,baj->ba", X, np.linalg.inv(B), X))
    assert np.max(np.abs(g.imag)) < IMAG
    assert np.max(np.abs(g.real - want)) < 2e-3


def test_nufft2_adjoint_against_the_exact_sum():
    sc = grangeat.Scan(16, 24, 32)
    om = grangeat.polar_omega(sc)
    rng = np.random.default_rng(3)
    c = rng.standard_normal(len(om)) + 1j * rng.standard_normal(len(om))
    a = grangeat.nufft2_adjoint(c, om, sc.n, sc.J, sc.beta)
    b = grangeat.nudft2_adjoint(c, om, sc.n)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 2e-4


@pytest.mark.parametrize("n_alpha,n", [(64, 64), (128, 64), (96, 48)])
@pytest.mark.parametrize("blob", ["centre", "off-axis"])
def test_projections_of_a_gaussian(n_alpha, n, blob):
    # closed-form umbrella values -> the whole step -> closed-form cone-beam
    # line integrals; the residual is the O(dk^4) quadrature error in k
    c, cov = (C0, COV) if blob == "centre" else (C_OFF, COV_OFF)
    sc = grangeat.Scan(32, n_alpha, n)
    n_proj = 3
    X = grangeat.projections(_umbrella_values(sc, n_proj, c, cov), sc)
    assert np.max(np.abs(X.imag)) < IMAG * np.max(np.abs(X))
    for k in range(n_proj):
        ref = _closed_projection(sc, k, n_proj, c, cov)
        assert np.max(np.abs(X[k].real - ref)) < 1.5e-3 * ref.max()


def _gauss_err(c=C_OFF, cov=COV_OFF):
    sc = grangeat.Scan(32, 64, 64)
    X = grangeat.projections(_umbrella_values(sc, 1, c, cov), sc)[0].real
    ref = _closed_projection(sc, 0, 1, c, cov)
    return np.max(np.abs(X - ref)) / ref.max()


def test_detects_missing_postweight(monkeypatch):
    assert _gauss_err() < 1e-3
    monkeypatch.setattr(grangeat, "depostweight", lambda U, sc: -np.asarray(U, dtype=complex))
    assert _gauss_err() > 3e-3


def test_detects_missing_preweight(monkeypatch):
    monkeypatch.setattr(grangeat, "depreweight", lambda g, sc: g)
    assert _gauss_err() > 3e-3


def test_detects_dc_weight_of_a_midpoint_rule(monkeypatch):
    # dk^2 / 4 (the ramp's integral over the k = 0 bin) instead of the
    # Euler-Maclaurin dk^2 / 6 of the trapezoidal rule
    orig = grangeat.radial_spectra

    def quarter(p, sc):
        c = orig(p, sc)
        c[:, sc.n] *= 6.0 / 4.0
        return c
    assert _gauss_err(C0, COV) < 1e-3
    monkeypatch.setattr(grangeat, "radial_spectra", quarter)
    assert _gauss_err(C0, COV) > 2e-3


def test_detects_flipped_filter_sign(monkeypatch):
    orig = grangeat.radial_spectra

    def flipped(p, sc):
        c = orig(p, sc)
        dc = c[:, sc.n].copy()
        c = -c
        c[:, sc.n] = dc
        return c
    monkeypatch.setattr(grangeat, "radial_spectra", flipped)
    assert _gauss_err() > 1e-1

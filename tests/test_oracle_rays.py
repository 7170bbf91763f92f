"""Pins of the oracle's ray propagation (Sec. 2.2, App. B-D) against the
paper's identities and limits."""
import numpy as np
import pytest

from oracle import healpix as hp
from oracle import rays
from oracle.mg import basis

KS = [-2e-7, 0.0, 3e-7]


@pytest.mark.parametrize("K", KS)
def test_distance_identities(K):
    """D_ac = (D_a D_bc + D_ab D_c)/D_b and D_ad = (D_ac D_bd - D_ab D_cd)/D_bc
    (App. C, App. D), with D_ab = r(chi_b - chi_a)."""
    rng = np.random.default_rng(1)
    D = lambda a, b: rays.r_of_chi(b - a, K)
    for _ in range(50):
        a, b, c, d = np.sort(rng.uniform(100, 3000, 4))
        assert np.isclose(D(a, c), (D(0, a) * D(b, c) + D(a, b) * D(0, c)) / D(0, b), rtol=1e-12)
        assert np.isclose(D(a, d), (D(a, c) * D(b, d) - D(a, b) * D(c, d)) / D(b, c), rtol=1e-10)


def test_negative_curvature_branch():
    K, chi = -4e-7, 1500.0
    assert np.isclose(rays.r_of_chi(chi, K), np.sinh(np.sqrt(-K) * chi) / np.sqrt(-K))
    assert rays.r_of_chi(chi, K) > chi > rays.r_of_chi(chi, -K)


def test_chi_of_z():
    z = np.array([0.1, 1.0, 3.0])
    ref = 2 * 2997.92458 * (1 - 1 / np.sqrt(1 + z))     # Omega_m = 1 closed form
    assert np.allclose(rays.chi_of_z(z, omega_m=1.0), ref, rtol=1e-12)
    assert abs(rays.chi_of_z(1.5, omega_m=0.3)[0] - 3054.70) < 0.01


@pytest.mark.parametrize("K", KS)
def test_recurrence_equals_direct_sum(K):
    """eq. Atraj == eq. Atrajold (App. C)."""
    rng = np.random.default_rng(2)
    chi = np.cumsum(rng.uniform(50, 200, 13))
    Us = [rng.normal(size=(2, 2)) * 0.05 for _ in range(12)]
    a = rays.jacobian_recurrence(chi, Us, K)
    b = rays.jacobian_direct_sum(chi, Us, K)
    for x, y in zip(a, b):
        assert np.allclose(x, y, atol=1e-13)


@pytest.mark.parametrize("K", KS)
def test_galaxy_interpolation_identity(K):
    """eq. gatraj with A_{n+1} from eq. Atraj equals eq. truegatraj (App. D)."""
    rng = np.random.default_rng(3)
    chi = np.cumsum(rng.uniform(80, 150, 8))
    Us = [rng.normal(size=(2, 2)) * 0.05 for _ in range(7)]
    A = rays.jacobian_recurrence(chi, Us, K)
    D = lambda a, b: rays.r_of_chi(b - a, K)
    for n in range(1, 6):
        chig = rng.uniform(chi[n], chi[n + 1])
        w = rays.galaxy_weight(chi, n + 1, chig, K)
        ga = (1 - w) * A[n] + w * A[n + 1]
        t = D(0, chi[n]) / D(0, chig) * D(chi[n - 1], chig) / D(chi[n - 1], chi[n])
        true = (1 - t) * A[n - 1] + t * A[n] - D(chi[n], chig) / D(0, chig) * Us[n] @ A[n]
        assert np.allclose(ga, true, atol=1e-13)


def _unit(th, ph):
    return hp.vec(np.cos(th), ph)


def test_transport_trivial_paths():
    for (a, b) in [((0.7, 1.1), (0.9, 1.1)),            # along a meridian
                   ((np.pi / 2, 0.2), (np.pi / 2, 0.9)),  # along the equator
                   ((1.3, 2.0), (1.3, 2.0))]:
        M = rays.transport_matrix(_unit(*a), _unit(*b))
        assert np.allclose(M, np.eye(2), atol=1e-14)
    M = rays.transport_matrix(_unit(0.4, 0.1), _unit(1.9, 2.5))
    assert np.allclose(M @ M.T, np.eye(2), atol=1e-14)
    assert np.isclose(np.linalg.det(M), 1.0)


def test_transport_holonomy_is_spherical_excess():
    """Transporting around a geodesic triangle rotates a vector by the
    enclosed spherical excess and a rank-2 tensor's traceless part by twice
    that (App. B)."""
    P = [_unit(0.6, 0.3), _unit(1.4, 0.2), _unit(1.1, 1.3)]
    M = np.eye(2)
    for k in range(3):
        M = rays.transport_matrix(P[k], P[(k + 1) % 3]) @ M
    a, b, c = P
    excess = 2 * np.arctan2(abs(a @ np.cross(b, c)), 1 + a @ b + b @ c + c @ a)
    ang = np.arctan2(M[1, 0], M[0, 0])
    assert np.isclose(abs(ang), excess, atol=1e-12)
    T = np.array([[0.3, 0.1], [0.1, -0.3]])
    T2 = M @ T @ M.T
    ang2 = np.arctan2(T2[0, 1], T2[0, 0]) - np.arctan2(T[0, 1], T[0, 0])
    assert np.isclose(np.mod(abs(ang2), 2 * np.pi), 2 * excess, atol=1e-12) or \
        np.isclose(2 * np.pi - np.mod(abs(ang2), 2 * np.pi), 2 * excess, atol=1e-12)


def test_small_angle_limit_and_sign():
    """One plane, constant gradient eps theta-hat: the angular position on
    the next plane moves by -(D_01/D_1) eps theta-hat (eq. disclighttraj):
    rays turn toward -grad psi."""
    chi = np.array([1000.0, 1600.0])
    for eps in (1e-4, 1e-5):
        r = rays.Ray(1.2, 0.4)
        rays.ray_step(r, chi, 0, np.array([eps, 0.5 * eps]), np.zeros((2, 2)))
        th, ph = hp.vec2ang(r.n)
        et, ep = basis(np.cos(1.2), 0.4)
        dv = r.n - _unit(1.2, 0.4)
        shift = np.array([dv @ et, dv @ ep])
        expect = -(600.0 / 1600.0) * np.array([eps, 0.5 * eps])
        assert np.allclose(shift, expect, atol=5 * eps * eps)


def test_born_single_plane_has_no_rotation():
    chi = np.array([800.0, 1200.0])
    r = rays.Ray(0.9, 5.0)
    U = np.array([[0.02, -0.013], [-0.013, -0.007]])
    rays.ray_step(r, chi, 0, np.array([3e-4, -2e-4]), U)
    assert abs(r.A[0, 1] - r.A[1, 0]) < 1e-15
    assert np.allclose(r.A_prev, np.eye(2), atol=1e-15)
    # and the first step is A^(1) = I - D_01/D_1 U up to transport
    M = rays.transport_matrix(_unit(0.9, 5.0), r.n)
    assert np.allclose(M.T @ r.A @ M, np.eye(2) - 0.4 / 1.2 * U / 1.0 * (1200 / 1200), atol=1e-14)


def test_ray_step_matches_recurrence_for_tiny_deflections():
    rng = np.random.default_rng(4)
    chi = np.cumsum(rng.uniform(100, 200, 7))
    Us = [rng.normal(size=(2, 2)) * 0.03 for _ in range(6)]
    Us = [0.5 * (U + U.T) for U in Us]
    r = rays.Ray(1.0, 1.0)
    for m in range(6):
        rays.ray_step(r, chi, m, np.zeros(2), Us[m])
    ref = rays.jacobian_recurrence(chi, Us)
    assert np.allclose(r.A, ref[-1], atol=1e-14)
    assert np.allclose(r.A_prev, ref[-2], atol=1e-14)


def closed_form_fields(nside, which):
    """Gradient and covariant Hessian of psi = z = cos(theta) or
    psi = x = sin(theta) cos(phi) at the RING pixel centres, by hand: for
    l = 1 the covariant Hessian is -psi times the metric."""
    z, ph, s = hp.pix2ang_ring(nside, np.arange(12 * nside * nside))
    if which == "z":
        psi, g = z, np.stack([-s, 0.0 * s])
    else:
        psi, g = s * np.cos(ph), np.stack([z * np.cos(ph), -np.sin(ph)])
    return g, np.stack([-psi, -psi, 0.0 * psi])


def exact_at(which, n):
    th, ph = hp.vec2ang(n)
    z, s = np.cos(th), np.sin(th)
    if which == "z":
        psi, g = z, np.array([-s, 0.0])
    else:
        psi, g = s * np.cos(ph), np.array([z * np.cos(ph), -np.sin(ph)])
    return g, -psi * np.eye(2)


def test_pixel_field_at_pixel_centres_is_exact():
    N = 8
    g, U = closed_form_fields(N, "x")
    for p in (0, 3, 100, 383, 767):
        z, ph, s = hp.pix2ang_ring(N, np.array([p]))
        gi, Ui = rays.pixel_field_at(N, g, U, hp.vec(z[0], ph[0], s[0]))
        np.testing.assert_allclose(gi, g[:, p], atol=1e-14)
        np.testing.assert_allclose(Ui, [[U[0, p], U[2, p]], [U[2, p], U[1, p]]], atol=1e-14)


@pytest.mark.parametrize("which", ["z", "x"])
def test_pixel_field_at_converges_with_transport(which):
    """Off-centre points: the interpolation error of the closed-form fields
    falls as Nside^-2 away from the poles (at least 3x per doubling) and at
    least as Nside^-1 inside the polar caps above the first ring, where the
    public package's scheme bilinearly joins four pixels 90 degrees apart
    through a virtual pole (at least 1.8x per doubling).  psi = x has a
    gradient whose (theta-hat, phi-hat) components turn with phi, at an
    O(1) rate near the poles, so an interpolation of the components without
    the transport would not converge there."""
    rng = np.random.default_rng(3)
    mid = hp.vec(rng.uniform(-0.9, 0.9, 40), rng.uniform(0, 2 * np.pi, 40))
    zc = np.concatenate([rng.uniform(0.995, 0.99999, 20), -rng.uniform(0.995, 0.99999, 20)])
    cap = hp.vec(zc, rng.uniform(0, 2 * np.pi, zc.size))
    errs = {"mid": [], "cap": []}
    for N in (16, 32, 64):
        g, U = closed_form_fields(N, which)
        for name, pts in (("mid", mid), ("cap", cap)):
            e = 0.0
            for n in pts:
                gi, Ui = rays.pixel_field_at(N, g, U, n)
                ge, Ue = exact_at(which, n)
                e = max(e, np.abs(gi - ge).max(), np.abs(Ui - Ue).max())
            errs[name].append(e)
    m, c = errs["mid"], errs["cap"]
    assert m[1] < m[0] / 3 and m[2] < m[1] / 3 and m[2] < 2e-4, errs
    assert c[1] < c[0] / 1.8 and c[2] < c[1] / 1.8 and c[2] < 5e-3, errs

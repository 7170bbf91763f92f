"""Galaxy images by the grid search, for the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

Sec. 2.3 and Sec. 3.3 of the paper: the rays start at the HEALPix pixel
centres of the image plane, which are joined into triangles covering the
sphere.  The ray tracing maps each image-plane triangle to the triangle of
the same three rays on the galaxy's source plane.  A triangle whose source
triangle contains the galaxy gives the image: barycentric coordinates of the
galaxy in the source triangle, computed in the plane tangent to the sphere at
the galaxy's source position (Press et al. 2007, Sec. 21.3), and the same
coordinates applied to the image-plane vertices.  The rays are moved from the
last lens plane to the galaxy's own distance first, with no further
deflection, taking the root of eq. posprop of least |lambda| (App. D).  The
Jacobian at the image is the HEALPix four-point interpolation of the ray
Jacobians, each parallel transported to the image position (App. B), and
combined over the last two planes by eq. gatraj.

Readings (the paper shows the triangles only in a figure):
* triangles join consecutive rings: between rings A and B the pixel centres
  are merged in azimuth, and each step of the merge adds the triangle of the
  current pair and the next vertex (A first on equal azimuth, which HEALPix
  rings never produce); the four pixels of each polar ring close the polar
  caps with two triangles;
* tangent-plane coordinates are the gnomonic projection about the galaxy,
  P(n) = n / (n . g), so an undeflected ray grid returns the source itself;
  the image is normalise(sum_i b_i P(n_i^image));
* a galaxy is inside a triangle when its three barycentric coordinates are
  >= 0; the first containing triangle in the search order (bands from north
  to south, then the merge order) is kept.
"""
import numpy as np

from . import healpix as hp
from .rays import r_of_chi, transport_matrix


# --------------------------------------------------------------------------
# ring structure and the triangles
# --------------------------------------------------------------------------
def ring_info(nside, q):
    """(first pixel, pixels, shift s) of 0-based ring q: pixel j of the ring
    sits at azimuth 2 pi (j + s / 2) / n."""
    N = nside
    i = q + 1
    if i < N:
        return 2 * i * (i - 1), 4 * i, 1
    if i <= 3 * N:
        return 2 * N * (N - 1) + 4 * N * (i - N), 4 * N, 1 if (i - N) % 2 == 0 else 0
    ip = 4 * N - i
    return 12 * N * N - 2 * ip * (ip + 1), 4 * ip, 1


def _pred(j_next, na, sa, nb, sb):
    """Index on ring B of the last vertex before vertex j_next of ring A in
    azimuth (cyclic): the largest k with (2k + sb) na < (2 j + sa) nb, in
    integers (no two vertices of adjacent HEALPix rings share an azimuth)."""
    X = (2 * np.asarray(j_next, dtype=np.int64) + sa) * nb - sb * na
    k = -((-X) // (2 * na)) - 1          # ceil(X / 2na) - 1
    return k % nb


def band_triangles(nside, q):
    """Triangles (rows of three RING pixel indices, counter-clockwise seen
    from outside) between ring q and ring q + 1 (q = -1: the north cap;
    q = 4 nside - 2: the south cap)."""
    nring = 4 * nside - 1
    if q == -1 or q == nring - 1:
        f, n, _ = ring_info(nside, 0 if q == -1 else nring - 1)
        p = f + np.arange(4)
        if q == -1:
            return np.array([[p[0], p[1], p[2]], [p[0], p[2], p[3]]], dtype=np.int64)
        return np.array([[p[0], p[2], p[1]], [p[0], p[3], p[2]]], dtype=np.int64)
    fa, na, sa = ring_info(nside, q)
    fb, nb, sb = ring_info(nside, q + 1)
    j = np.arange(na, dtype=np.int64)
    jn = (j + 1) % na
    ta = np.stack([fa + j, fb + _pred(jn, na, sa, nb, sb), fa + jn], axis=1)
    k = np.arange(nb, dtype=np.int64)
    kn = (k + 1) % nb
    tb = np.stack([fb + k, fb + kn, fa + _pred(kn, nb, sb, na, sa)], axis=1)
    return np.concatenate([ta, tb])


def all_triangles(nside):
    """Every triangle of the image-plane covering, bands north to south."""
    return np.concatenate([band_triangles(nside, q) for q in range(-1, 4 * nside - 1)])


def spherical_area(a, b, c):
    """Signed area of the spherical triangle of unit vectors (rows) a, b, c
    (positive when a, b, c run counter-clockwise seen from outside)."""
    num = np.einsum("ij,ij->i", a, np.cross(b, c))
    den = 1 + np.einsum("ij,ij->i", a, b) + np.einsum("ij,ij->i", b, c) + \
        np.einsum("ij,ij->i", c, a)
    return 2 * np.arctan2(num, den)


def pixel_vectors(nside, pix):
    z, ph, s = hp.pix2ang_ring(nside, np.asarray(pix))
    return hp.vec(z, ph, s)


# --------------------------------------------------------------------------
# the search
# --------------------------------------------------------------------------
def barycentric(g, v1, v2, v3):
    """Barycentric coordinates of the unit vector g in the triangle (v1, v2,
    v3) after gnomonic projection onto the plane tangent at g."""
    P = [v / np.dot(v, g) - g for v in (v1, v2, v3)]
    e1, e2 = P[1] - P[0], P[2] - P[0]
    r = -P[0]                                   # the galaxy projects to 0
    m = np.array([[e1 @ e1, e1 @ e2], [e1 @ e2, e2 @ e2]])
    rhs = np.array([r @ e1, r @ e2])
    b2, b3 = np.linalg.solve(m, rhs)
    return np.array([1.0 - b2 - b3, b2, b3])


def propagate(n_ray, beta, chi_from, chi_to):
    """Unit position of a ray moved along beta from radius chi_from to
    chi_to, the root of |x + lambda beta| = chi_to of least |lambda|."""
    x = chi_from * n_ray
    b = x @ beta
    q = chi_to * chi_to - chi_from * chi_from
    lam = q / (b + np.sqrt(b * b + q))
    y = x + lam * beta
    return y / np.linalg.norm(y)


def candidate_bands(nside, g, radius):
    """Bands whose rings come within `radius` (rad) of the unit vector g,
    with a margin of one ring."""
    rt = hp.ring_table(nside)
    th = np.arccos(np.clip(rt["z"], -1, 1))
    tg = np.arccos(np.clip(g[2], -1, 1))
    near = np.nonzero(np.abs(th - tg) <= radius + 2.5 / nside)[0]
    lo, hi = max(near.min() - 1, -1), min(near.max(), 4 * nside - 2)
    return range(lo, hi + 1)


def find_image(nside, g, src_of, radius):
    """Image of the galaxy at unit source position g: src_of(pixels) gives the
    source-plane unit vectors of the rays of RING pixels (rows).  Returns
    (image unit vector, triangle pixels, barycentric coordinates) or None."""
    for q in candidate_bands(nside, g, radius):
        tri = band_triangles(nside, q)
        # triangles with a vertex within the radius (image plane) of g
        v = pixel_vectors(nside, tri.ravel()).reshape(-1, 3, 3)
        close = np.any(v @ g >= np.cos(radius + 2.0 / nside), axis=1)
        for t in np.nonzero(close)[0]:
            s = src_of(tri[t])
            if np.any(s @ g <= 0):
                continue
            b = barycentric(g, s[0], s[1], s[2])
            if np.all(b >= 0.0):
                vi = v[t]
                img = sum(b[i] * vi[i] / (vi[i] @ g) for i in range(3))
                return img / np.linalg.norm(img), tri[t], b
    return None


def image_jacobian(nside, img, A_ray, Ap_ray, n_ray, w):
    """eq. gatraj at the image: the four-point HEALPix interpolation at img of
    the ray Jacobians A^(k) (A_ray) and A^(k-1) (Ap_ray), callables of a RING
    pixel returning a 2 x 2 matrix, each transported from its ray's position
    n_ray(pixel) to img (App. B), then (1 - w) A^(k-1) + w A^(k)."""
    th, ph = hp.vec2ang(img)
    pix, wt = hp.interp_weights(nside, np.array([th]), np.array([ph]))
    A = np.zeros((2, 2))
    Ap = np.zeros((2, 2))
    for c in range(4):
        p = int(pix[c, 0])
        M = transport_matrix(n_ray(p), img)
        A += wt[c, 0] * (M @ A_ray(p) @ M.T)
        Ap += wt[c, 0] * (M @ Ap_ray(p) @ M.T)
    return (1 - w) * Ap + w * A


def shell_weight(chi_km1, chi_k, chi_g, K=0.0):
    """w of eq. gatraj: D_k D_{k-1,g} / (D_g D_{k-1,k})."""
    D = lambda a, b: float(r_of_chi(b - a, K))
    return D(0, chi_k) * D(chi_km1, chi_g) / (D(0, chi_g) * D(chi_km1, chi_k))


def galaxy_images(nside, rays, chi, k, gal_theta, gal_phi, gal_chi, radius, K=0.0):
    """The grid search for galaxies of shell k after the rays were moved
    through plane k - 1.  rays: dict of NESTED-order arrays theta, phi
    (current angular position at chi_k), beta [3][n], A, A_prev [4][n].
    Returns per galaxy (found, image theta, image phi, A_g [2][2]) for the
    galaxies in the shell (None for the others)."""
    chi = np.asarray(chi, dtype=np.float64)
    edges = np.concatenate([[0.0], 0.5 * (chi[:-1] + chi[1:])])
    hi = edges[k + 1] if k + 1 < len(edges) else np.inf

    def r2n(p):
        return int(hp.ring2nest_pix(nside, np.array([p]))[0])

    def nvec(i):
        return hp.vec(np.cos(rays["theta"][i]), rays["phi"][i])

    out = []
    for th, ph, cg in zip(gal_theta, gal_phi, gal_chi):
        if not (edges[k] <= cg < hi):
            out.append(None)
            continue
        g = hp.vec(np.cos(th), ph)
        if k == 0:
            out.append((True, th, ph, np.eye(2)))
            continue

        def src_of(pix):
            res = []
            for p in pix:
                i = r2n(int(p))
                b = np.array([rays["beta"][0][i], rays["beta"][1][i], rays["beta"][2][i]])
                res.append(propagate(nvec(i), b, chi[k], cg))
            return np.array(res)

        found = find_image(nside, g, src_of, radius)
        if found is None:
            out.append((False, np.nan, np.nan, np.full((2, 2), np.nan)))
            continue
        img = found[0]
        w = shell_weight(chi[k - 1], chi[k], cg, K)
        Aq = lambda p: np.asarray(rays["A"][:, r2n(p)], dtype=np.float64).reshape(2, 2)
        Apq = lambda p: np.asarray(rays["A_prev"][:, r2n(p)], dtype=np.float64).reshape(2, 2)
        Ag = image_jacobian(nside, img, Aq, Apq, lambda p: nvec(r2n(p)), w)
        ti, pi = hp.vec2ang(img)
        out.append((True, ti, pi, Ag))
    return out

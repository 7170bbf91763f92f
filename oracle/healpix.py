"""HEALPix pixelization for the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import this module.

The paper places rays on HEALPix cell centres, groups them into bundles of a
coarser NESTED resolution with a bit shift (Sec. 3.1), runs the SHT on a
HEALPix grid (Sec. 3.2) and uses the public package's linear interpolation to
carry the SHT potential onto the multigrid patches (Sec. 3.2).  The
pixelization itself is the published one (Gorski et al. 2005, ApJ 622, 759);
it is restated here from its definition:

* 12 N^2 equal-area pixels (Sec. 4.1, footnote: area 4 pi / (12 N^2)),
  centres on 4N-1 iso-latitude rings;
* RING order numbers pixels ring by ring, west to east from phi = 0;
* NESTED order numbers the 12 base faces, then interleaves the bits of the
  (x, y) position inside a face, so pixel p at N has children 4p..4p+3 at 2N.

All arithmetic is float64 numpy; every function accepts arrays.
"""
import numpy as np

# Base-face layout: ring-number offset (in units of N) and phi offset (in
# units of pi/4 per ring-pixel quarter) of each of the 12 base faces.
_JRLL = np.array([2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4], dtype=np.int64)
_JPLL = np.array([1, 3, 5, 7, 0, 2, 4, 6, 1, 3, 5, 7], dtype=np.int64)


def npix(nside):
    return 12 * nside * nside


def ring_table(nside):
    """Per-ring geometry for rings i = 1 .. 4N-1 (returned 0-based).

    Returns dict of arrays: z (cos theta), sint (sin theta), n (pixels in
    ring), first (RING index of the ring's first pixel), phi0 (longitude of
    the first pixel centre), shifted (phi0 != 0).
    """
    N = nside
    i = np.arange(1, 4 * N, dtype=np.int64)
    z = np.empty(i.size)
    one_minus_z = np.empty(i.size)
    n = np.empty(i.size, dtype=np.int64)
    first = np.empty(i.size, dtype=np.int64)
    shifted = np.ones(i.size, dtype=bool)
    north = i < N
    belt = (i >= N) & (i <= 3 * N)
    south = i > 3 * N
    # north polar cap: z = 1 - i^2/(3N^2), 4i pixels
    ii = i[north].astype(np.float64)
    one_minus_z[north] = ii * ii / (3.0 * N * N)
    z[north] = 1.0 - one_minus_z[north]
    n[north] = 4 * i[north]
    first[north] = 2 * i[north] * (i[north] - 1)
    # equatorial belt: z = 4/3 - 2i/(3N), 4N pixels, every other ring shifted
    ib = i[belt]
    z[belt] = (4.0 * N - 2.0 * ib) / (3.0 * N)
    one_minus_z[belt] = 1.0 - z[belt]
    n[belt] = 4 * N
    first[belt] = 2 * N * (N - 1) + 4 * N * (ib - N)
    shifted[belt] = ((ib - N) % 2) == 0
    # south polar cap: mirror of the north cap
    ip = 4 * N - i[south]
    ipf = ip.astype(np.float64)
    one_plus_z = ipf * ipf / (3.0 * N * N)
    z[south] = one_plus_z - 1.0
    one_minus_z[south] = 2.0 - one_plus_z
    n[south] = 4 * ip
    first[south] = 12 * N * N - 2 * ip * (ip + 1)
    # sin(theta) = sqrt((1-z)(1+z)), formed from the exact 1-z in the caps
    sint = np.sqrt(one_minus_z * (1.0 + z))
    sint[south] = np.sqrt(one_plus_z * (2.0 - one_plus_z))
    phi0 = np.where(shifted, np.pi / n, 0.0)
    return dict(z=z, sint=sint, n=n, first=first, phi0=phi0, shifted=shifted,
                theta=np.arctan2(sint, z))


def pix2ring(nside, p):
    """0-based ring number of RING-ordered pixel(s) p."""
    rt = ring_table(nside)
    return np.searchsorted(rt["first"], np.asarray(p), side="right") - 1


def pix2ang_ring(nside, p):
    """(z, phi, sin theta) of RING pixel centres."""
    rt = ring_table(nside)
    p = np.asarray(p, dtype=np.int64)
    r = np.searchsorted(rt["first"], p, side="right") - 1
    j = p - rt["first"][r]
    phi = rt["phi0"][r] + 2.0 * np.pi * j / rt["n"][r]
    return rt["z"][r], phi, rt["sint"][r]


def _spread_bits(v):
    """Place bit k of v at bit 2k."""
    v = np.asarray(v, dtype=np.int64)
    out = np.zeros_like(v)
    for k in range(31):
        out |= ((v >> k) & 1) << (2 * k)
    return out


def _compact_bits(v):
    """Inverse of _spread_bits: gather the even bits of v."""
    v = np.asarray(v, dtype=np.int64)
    out = np.zeros_like(v)
    for k in range(31):
        out |= ((v >> (2 * k)) & 1) << k
    return out


def nest2xyf(nside, p):
    p = np.asarray(p, dtype=np.int64)
    face = p // (nside * nside)
    q = p % (nside * nside)
    return _compact_bits(q), _compact_bits(q >> 1), face


def xyf2nest(nside, ix, iy, face):
    return np.asarray(face, dtype=np.int64) * nside * nside + \
        _spread_bits(ix) + (_spread_bits(iy) << 1)


def xyf2ring(nside, ix, iy, face):
    """RING index of the pixel at (ix, iy) on base face `face`."""
    N = nside
    ix = np.asarray(ix, dtype=np.int64)
    iy = np.asarray(iy, dtype=np.int64)
    face = np.asarray(face, dtype=np.int64)
    jr = _JRLL[face] * N - ix - iy - 1          # 1-based ring number
    nr = np.where(jr < N, jr, np.where(jr > 3 * N, 4 * N - jr, N))
    kshift = np.where((jr >= N) & (jr <= 3 * N), (jr - N) & 1, 0)
    jp = (_JPLL[face] * nr + ix - iy + 1 + kshift) // 2
    jp = np.where(jp > 4 * N, jp - 4 * N, jp)
    jp = np.where(jp < 1, jp + 4 * nr, jp)
    first = np.where(jr < N, 2 * jr * (jr - 1),
                     np.where(jr > 3 * N, 12 * N * N - 2 * nr * (nr + 1),
                              2 * N * (N - 1) + 4 * N * (jr - N)))
    return first + jp - 1


def nest2ring(nside, p):
    ix, iy, f = nest2xyf(nside, p)
    return xyf2ring(nside, ix, iy, f)


def ring2nest(nside, p):
    """Inverse permutation of nest2ring (built by brute force: oracle-sized)."""
    allnest = np.arange(npix(nside), dtype=np.int64)
    inv = np.empty_like(allnest)
    inv[nest2ring(nside, allnest)] = allnest
    return inv[np.asarray(p, dtype=np.int64)]


def ring2nest_pix(nside, p):
    """NESTED index of the RING pixels p, without the full permutation: the
    NESTED pixel that holds each RING pixel's centre (a centre lies half a
    pixel inside its own pixel)."""
    z, phi, _ = pix2ang_ring(nside, np.asarray(p, dtype=np.int64))
    return ang2pix_nest(nside, z, phi)


def pix2ang_nest(nside, p):
    return pix2ang_ring(nside, nest2ring(nside, p))


def ang2pix_nest(nside, z, phi):
    """NESTED pixel containing the direction (z = cos theta, phi)."""
    N = nside
    z = np.asarray(z, dtype=np.float64)
    za = np.abs(z)
    tt = np.mod(np.asarray(phi, dtype=np.float64), 2.0 * np.pi) * (2.0 / np.pi)
    tt = np.where(tt >= 4.0, tt - 4.0, tt)
    out = np.empty(z.shape, dtype=np.int64)
    eq = za <= 2.0 / 3.0
    # equatorial region: pixel edges are straight lines in (z, phi)
    t1 = N * (0.5 + tt[eq])
    t2 = N * (z[eq] * 0.75)
    jp = np.floor(t1 - t2).astype(np.int64)
    jm = np.floor(t1 + t2).astype(np.int64)
    ifp = jp // N
    ifm = jm // N
    face = np.where(ifp == ifm, ifp | 4, np.where(ifp < ifm, ifp, ifm + 8))
    ix = jm & (N - 1)
    iy = N - (jp & (N - 1)) - 1
    out[eq] = xyf2nest(N, ix, iy, face)
    # polar caps
    pc = ~eq
    ntt = np.minimum(3, np.floor(tt[pc]).astype(np.int64))
    tp = tt[pc] - ntt
    tmp = N * np.sqrt(3.0 * (1.0 - za[pc]))
    jp = np.minimum(np.floor(tp * tmp).astype(np.int64), N - 1)
    jm = np.minimum(np.floor((1.0 - tp) * tmp).astype(np.int64), N - 1)
    north = z[pc] >= 0
    face = np.where(north, ntt, ntt + 8)
    ix = np.where(north, N - jm - 1, jp)
    iy = np.where(north, N - jp - 1, jm)
    out[pc] = xyf2nest(N, ix, iy, face)
    return out


def vec(z, phi, sint=None):
    """Unit vector(s) for (z = cos theta, phi); shape (..., 3)."""
    z = np.asarray(z, dtype=np.float64)
    if sint is None:
        sint = np.sqrt((1.0 - z) * (1.0 + z))
    return np.stack([sint * np.cos(phi), sint * np.sin(phi), z], axis=-1)


def vec2ang(v):
    """(theta, phi in [0, 2pi)) of vector(s) v (..., 3)."""
    v = np.asarray(v, dtype=np.float64)
    theta = np.arctan2(np.hypot(v[..., 0], v[..., 1]), v[..., 2])
    phi = np.arctan2(v[..., 1], v[..., 0])
    phi = np.where(phi < 0, phi + 2.0 * np.pi, phi)
    return theta, phi


def degrade_nest_mean(nside_in, nside_out, m_nest):
    """Mean of the NESTED children (mass-conserving degrade; Sec. 3.2 states
    that the binning conserves mass exactly).  Input and output NESTED."""
    k = (nside_in // nside_out) ** 2
    return np.asarray(m_nest).reshape(npix(nside_out), k).mean(axis=1)


def interp_weights(nside, theta, phi):
    """Four RING pixels and bilinear weights for a direction (the public
    package's linear interpolation used by Sec. 3.2 and 3.3): bracket theta
    between two rings, bracket phi inside each ring, weight linearly in each.
    Above the first ring (below the last) the missing ring is replaced by a
    virtual pole whose value is the mean of that ring's four pixels.
    Returns (pix[4, n], w[4, n])."""
    rt = ring_table(nside)
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    phi = np.atleast_1d(np.asarray(phi, dtype=np.float64))
    nring = rt["n"].size
    th = rt["theta"]
    ir1 = np.searchsorted(th, theta, side="right") - 1   # -1: above ring 0
    ir1 = np.minimum(ir1, nring - 1)
    pix = np.zeros((4, theta.size), dtype=np.int64)
    w = np.zeros((4, theta.size))

    def ring_pair(r, ph):
        nr = rt["n"][r]
        t = (ph - rt["phi0"][r]) * nr / (2.0 * np.pi)
        fl = np.floor(t)
        wphi = t - fl
        i1 = np.mod(fl.astype(np.int64), nr)
        i2 = np.mod(i1 + 1, nr)
        return rt["first"][r] + i1, rt["first"][r] + i2, wphi

    mid = (ir1 >= 0) & (ir1 < nring - 1)
    r1 = ir1[mid]
    r2 = r1 + 1
    a1, a2, wa = ring_pair(r1, phi[mid])
    b1, b2, wb = ring_pair(r2, phi[mid])
    wt = (theta[mid] - th[r1]) / (th[r2] - th[r1])
    pix[:, mid] = np.stack([a1, a2, b1, b2])
    w[:, mid] = np.stack([(1 - wt) * (1 - wa), (1 - wt) * wa,
                          wt * (1 - wb), wt * wb])

    north = ir1 < 0
    if np.any(north):
        b1, b2, wb = ring_pair(np.zeros(north.sum(), dtype=np.int64), phi[north])
        wt = theta[north] / th[0]
        # the other two pixels of ring 0 (4 pixels total): the pole value is
        # the mean of all four
        c1 = np.mod(b1 + 2, 4)
        c2 = np.mod(b2 + 2, 4)
        fac = (1.0 - wt) * 0.25
        pix[:, north] = np.stack([b1, b2, c1, c2])
        w[:, north] = np.stack([wt * (1 - wb) + fac, wt * wb + fac, fac, fac])
    south = ir1 >= nring - 1
    if np.any(south):
        r = np.full(south.sum(), nring - 1, dtype=np.int64)
        a1, a2, wa = ring_pair(r, phi[south])
        wt = (theta[south] - th[-1]) / (np.pi - th[-1])
        base = rt["first"][-1]
        c1 = base + np.mod(a1 - base + 2, 4)
        c2 = base + np.mod(a2 - base + 2, 4)
        fac = wt * 0.25
        pix[:, south] = np.stack([a1, a2, c1, c2])
        w[:, south] = np.stack([(1 - wt) * (1 - wa) + fac, (1 - wt) * wa + fac,
                                fac, fac])
    return pix, w


def interp(nside, m_ring, theta, phi):
    """Linear interpolation of a RING map at (theta, phi)."""
    pix, w = interp_weights(nside, theta, phi)
    return np.sum(np.asarray(m_ring)[pix] * w, axis=0)

"""Point sets of the HSMA oracle: wrapped positions, near image sets,
check points, and the quadrature on the auxiliary sphere.

Coordinates are centred: the box is [-L/2, L/2)^3 as in Sec. 2.1 (for the
slab, the dielectric interfaces sit at z = +-Lz/2).
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN_FRAC = (math.sqrt(5.0) - 1.0) / 2.0


def centre_and_wrap(pos, box_lo, box_len, periodic=(True, True, True)):
    """Shift to box-centred coordinates; wrap periodic axes into [-L/2, L/2)."""
    L = np.asarray(box_len, dtype=np.float64)
    x = np.asarray(pos, dtype=np.float64) - (np.asarray(box_lo, dtype=np.float64) + 0.5 * L)
    for k in range(3):
        if periodic[k]:
            x[:, k] -= L[k] * np.floor(x[:, k] / L[k] + 0.5)
    return x


# ---------------------------------------------------------------- images
def shifts_3d():
    """The 27 lattice shifts k in {-1,0,1}^3 (Eq. 3), kx slowest."""
    return np.array([(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)], dtype=np.float64)


def images_3d(x, q, L):
    """Near set S for the fully periodic system: every particle in the 27
    cells around (and including) the central box.  Returns sources (27N,3),
    charges (27N,) and, for particle i, the index of its own k=0 copy."""
    L = np.asarray(L, dtype=np.float64)
    ks = shifts_3d()
    src = (x[None, :, :] + (ks * L)[:, None, :]).reshape(-1, 3)
    qs = np.tile(q, len(ks))
    centre = 13  # k = (0,0,0)
    assert np.all(ks[centre] == 0)
    self_idx = centre * len(q) + np.arange(len(q))
    return src, qs, self_idx


def image_strengths(l: int, gamma_up: float, gamma_low: float):
    """Strength factors of the l-th upper and lower images (Eq. 4).

    The upper image of order l carries gamma_up^ceil(l/2) gamma_low^floor(l/2)
    and the lower image gamma_low^ceil(l/2) gamma_up^floor(l/2): the first
    reflection across the top interface must carry that interface's
    mismatch.  (The paper prints the two exponents the other way round;
    the two readings coincide when gamma_up = gamma_low.)"""
    c, f = (l + 1) // 2, l // 2
    return gamma_up ** c * gamma_low ** f, gamma_low ** c * gamma_up ** f


def images_2d(x, q, L, M, gamma_up, gamma_low, inplane=1):
    """Near set S for the slab: in-plane shifts k in {-inplane..inplane}^2,
    and for each the sources plus image layers l = 1..M above and below.
    The l-th image of z sits at (-1)^l z +- l Lz (Eq. 4)."""
    L = np.asarray(L, dtype=np.float64)
    n = len(q)
    blocks, charges = [], []
    rng = range(-inplane, inplane + 1)
    self_idx = None
    for a in rng:
        for b in rng:
            sh = np.array([a * L[0], b * L[1], 0.0])
            if a == 0 and b == 0:
                self_idx = sum(len(c) for c in charges) + np.arange(n)
            blocks.append(x + sh)
            charges.append(q.copy())
            for l in range(1, M + 1):
                gu, gl = image_strengths(l, gamma_up, gamma_low)
                sgn = -1.0 if l % 2 else 1.0
                up = x + sh
                up = up.copy()
                up[:, 2] = sgn * x[:, 2] + l * L[2]
                lo = (x + sh).copy()
                lo[:, 2] = sgn * x[:, 2] - l * L[2]
                blocks.append(up)
                charges.append(gu * q)
                blocks.append(lo)
                charges.append(gl * q)
    return np.concatenate(blocks), np.concatenate(charges), self_idx


# --------------------------------------------------------- check points
def _face_pairs(L, K, axes):
    """K check-point pairs on opposite box faces, round-robin over `axes`.

    Pair t lies on axis d = axes[t mod len(axes)]; with j = t div len(axes)
    and K_d pairs on that axis, its in-face coordinates are
    u = (j+1/2)/K_d - 1/2 and v = frac(j (sqrt5-1)/2) - 1/2 along the two
    other axes (in increasing order), scaled by their box lengths.
    x- sits on the face at -L_d/2, x+ = x- + L_d e_d."""
    L = np.asarray(L, dtype=np.float64)
    na = len(axes)
    xm = np.zeros((K, 3))
    axis = np.zeros(K, dtype=np.int64)
    for t in range(K):
        d = axes[t % na]
        j = t // na
        Kd = (K - (t % na) + na - 1) // na
        others = [a for a in range(3) if a != d]
        u = (j + 0.5) / Kd - 0.5
        jg = j * GOLDEN_FRAC
        v = (jg - math.floor(jg)) - 0.5
        xm[t, d] = -0.5 * L[d]
        xm[t, others[0]] = u * L[others[0]]
        xm[t, others[1]] = v * L[others[1]]
        axis[t] = d
    xp = xm.copy()
    xp[np.arange(K), axis] += L[axis]
    return xm, xp, axis


def check_pairs_3d(L, K):
    return _face_pairs(L, K, (0, 1, 2))


def check_pairs_2d(L, K):
    return _face_pairs(L, K, (0, 1))


def interface_grid(L, nz, top: bool):
    """nz x nz cell-centred points on the interface z = +Lz/2 (top) or -Lz/2;
    flattened with the x index slowest."""
    L = np.asarray(L, dtype=np.float64)
    gx = (np.arange(nz) + 0.5) * L[0] / nz - 0.5 * L[0]
    gy = (np.arange(nz) + 0.5) * L[1] / nz - 0.5 * L[1]
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    z = 0.5 * L[2] if top else -0.5 * L[2]
    return np.stack([X.ravel(), Y.ravel(), np.full(nz * nz, z)], axis=1)


def spectral_dtn(f, L, nz):
    """Apply T = DFT^-1 diag(|G|) DFT to grid samples f (nz*nz, ...) with
    G = 2 pi (m_x/Lx, m_y/Ly): the Dirichlet-to-Neumann map of a potential
    that decays away from the interface, for the periodic in-plane modes."""
    f = np.asarray(f, dtype=np.float64)
    shp = f.shape
    g = f.reshape((nz, nz) + shp[1:])
    m = np.fft.fftfreq(nz, d=1.0 / nz)
    gx = 2 * np.pi * m / L[0]
    gy = 2 * np.pi * m / L[1]
    G = np.sqrt(gx[:, None] ** 2 + gy[None, :] ** 2)
    G = G.reshape((nz, nz) + (1,) * (len(shp) - 1))
    out = np.fft.ifft2(G * np.fft.fft2(g, axes=(0, 1)), axes=(0, 1)).real
    return out.reshape(shp)


# ------------------------------------------------ surface quadrature
FIBONACCI = (1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144, 233, 377, 610, 987, 1597, 2584, 4181, 6765)


def zaremba_index(F: int, g: int) -> int:
    """min over nonzero dual-lattice vectors (h1,h2), h1 + g h2 = 0 mod F,
    of max(1,|h1|) max(1,|h2|) for the rank-1 lattice (k/F, k g/F)."""
    best = F  # (h1, h2) = (F, 0)
    for h2 in range(1, F // 2 + 1):
        h1 = (-g * h2) % F
        if h1 > F // 2:
            h1 -= F
        best = min(best, max(1, abs(h1)) * h2)
    return best


def lattice_generator(F: int, Fw: int = 0) -> int:
    """Generator of the rank-1 lattice: Fw if given; the preceding Fibonacci
    number if F is one (the Fibonacci lattice); else the smallest g in
    [1, F/2] that maximises the Zaremba index."""
    if Fw > 0:
        return Fw
    if F in FIBONACCI and F > 2:
        return FIBONACCI[FIBONACCI.index(F) - 1]
    best_g, best = 1, -1
    for g in range(1, F // 2 + 1):
        z = zaremba_index(F, g)
        if z > best:
            best, best_g = z, g
    return best_g


def _psi(t):
    return 10 * t ** 3 - 15 * t ** 4 + 6 * t ** 5


def _dpsi(t):
    return 30 * t ** 2 - 60 * t ** 3 + 30 * t ** 4


def surface_rule(F: int, R: float, rule: int = 0, Fw: int = 0):
    """Points y_k = R n_k, unit normals n_k and weights w_k on the sphere of
    radius R such that sum_k w_k f(y_k) ~ integral of f over the sphere.

    rule 0: periodised rank-1 lattice (the Fibonacci lattice when F is a
      Fibonacci number): t = k/F, theta = pi psi(t) with the Korobov
      polynomial psi(t) = 10t^3 - 15t^4 + 6t^5, phi = 2 pi frac(k g / F),
      w = R^2 sin(theta) pi psi'(t) 2 pi / F.
    rule 1: Gauss-Legendre in cos(theta) x trapezoid in phi; F = 2 n^2."""
    if rule == 0:
        g = lattice_generator(F, Fw)
        k = np.arange(F)
        t = k / F
        th = np.pi * _psi(t)
        ph = 2 * np.pi * ((k * g) % F) / F
        w = R * R * np.sin(th) * np.pi * _dpsi(t) * 2 * np.pi / F
    elif rule == 1:
        n = int(round(math.sqrt(F / 2)))
        if 2 * n * n != F:
            raise ValueError("rule 1 needs F = 2 n^2")
        ct, wt = np.polynomial.legendre.leggauss(n)
        th = np.repeat(np.arccos(ct), 2 * n)
        ph = np.tile(2 * np.pi * np.arange(2 * n) / (2 * n), n)
        w = R * R * np.repeat(wt, 2 * n) * (2 * np.pi / (2 * n))
    else:
        raise ValueError(rule)
    nrm = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=1)
    return R * nrm, nrm, w

"""Harmonic polynomial basis for the far-field series of Eq. (5).

The paper expands the potential of the charges outside the auxiliary sphere
as sum_{n<=P} sum_m A_n^m r^n Y_n^m, i.e. in the space of harmonic
polynomials of degree <= P.  The least-squares minimiser over that space
does not depend on which basis spans it, so the oracle uses its own family:
for each degree n it takes the null space of the Laplacian acting on the
homogeneous monomials x^a y^b z^c (a+b+c = n), and orthonormalises it on the
unit sphere.  The constant (n = 0) is left out: it is in the null space of
every fitting row (the potential is defined up to a constant).

All polynomials are in scaled coordinates xi = r / R.
"""
from __future__ import annotations

import functools

import numpy as np


@functools.lru_cache(maxsize=None)
def monomials(n: int):
    """Exponent triples (a, b, c) with a + b + c = n, in a fixed order."""
    return tuple((a, b, n - a - b) for a in range(n, -1, -1) for b in range(n - a, -1, -1))


def laplacian_matrix(n: int) -> np.ndarray:
    """Matrix of the Laplacian from degree-n to degree-(n-2) monomial coefficients."""
    src = monomials(n)
    if n < 2:
        return np.zeros((0, len(src)))
    dst = {m: i for i, m in enumerate(monomials(n - 2))}
    lap = np.zeros((len(dst), len(src)))
    for j, (a, b, c) in enumerate(src):
        if a >= 2:
            lap[dst[(a - 2, b, c)], j] += a * (a - 1)
        if b >= 2:
            lap[dst[(a, b - 2, c)], j] += b * (b - 1)
        if c >= 2:
            lap[dst[(a, b, c - 2)], j] += c * (c - 1)
    return lap


def _monomial_values(xi: np.ndarray, n: int) -> np.ndarray:
    e = np.array(monomials(n))
    return np.prod(xi[:, None, :] ** e[None, :, :], axis=2)


def _monomial_grads(xi: np.ndarray, n: int) -> np.ndarray:
    """d/dxi_k of every degree-n monomial: shape (npts, nmono, 3)."""
    e = np.array(monomials(n))
    out = np.zeros((xi.shape[0], e.shape[0], 3))
    for k in range(3):
        ek = e.copy()
        coef = ek[:, k].astype(np.float64)
        ek[:, k] = np.maximum(ek[:, k] - 1, 0)
        out[:, :, k] = coef[None, :] * np.prod(xi[:, None, :] ** ek[None, :, :], axis=2)
    return out


def _sphere_product_rule(order: int):
    """Gauss-Legendre in cos(theta) x trapezoid in phi, exact for polynomials
    of degree <= order on the unit sphere."""
    nt = order // 2 + 1
    nphi = order + 1
    ct, wt = np.polynomial.legendre.leggauss(nt)
    ph = 2 * np.pi * np.arange(nphi) / nphi
    st = np.sqrt(1 - ct ** 2)
    pts = np.stack([np.outer(st, np.cos(ph)).ravel(), np.outer(st, np.sin(ph)).ravel(),
                    np.repeat(ct, nphi)], axis=1)
    w = np.repeat(wt, nphi) * (2 * np.pi / nphi)
    return pts, w


@functools.lru_cache(maxsize=None)
def harmonic_basis(p: int):
    """Coefficient matrices C_n (nmono(n) x (2n+1)) for n = 1..p.

    Columns span the harmonic homogeneous polynomials of degree n and are
    orthonormal in L2 of the unit sphere."""
    pts, w = _sphere_product_rule(2 * p + 2)
    out = []
    for n in range(1, p + 1):
        lap = laplacian_matrix(n)
        nm = len(monomials(n))
        if lap.shape[0] == 0:
            C = np.eye(nm)
        else:
            _, s, vt = np.linalg.svd(lap)
            rank = int(np.sum(s > 1e-10 * s[0]))
            C = vt[rank:].T
        assert C.shape[1] == 2 * n + 1, (n, C.shape)
        V = _monomial_values(pts, n) @ C
        _, r = np.linalg.qr(np.sqrt(w)[:, None] * V)
        out.append(C @ np.linalg.inv(r))
    return tuple(out)


def nbasis(p: int) -> int:
    """Number of unknowns: (p+1)^2 - 1 (the constant is excluded)."""
    return (p + 1) ** 2 - 1


def degrees(p: int) -> np.ndarray:
    return np.concatenate([np.full(2 * n + 1, n) for n in range(1, p + 1)])


def values(r: np.ndarray, R: float, p: int) -> np.ndarray:
    """b_j(r) for every basis function j (npts x nbasis), r in physical units."""
    xi = np.asarray(r, dtype=np.float64).reshape(-1, 3) / R
    return np.concatenate([_monomial_values(xi, n) @ C for n, C in enumerate(harmonic_basis(p), 1)], axis=1)


def gradients(r: np.ndarray, R: float, p: int) -> np.ndarray:
    """grad_r b_j(r): shape (npts, nbasis, 3), physical units."""
    xi = np.asarray(r, dtype=np.float64).reshape(-1, 3) / R
    blocks = [np.einsum("pmk,mj->pjk", _monomial_grads(xi, n), C) for n, C in enumerate(harmonic_basis(p), 1)]
    return np.concatenate(blocks, axis=1) / R

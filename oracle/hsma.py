"""Plain FP64 HSMA (harmonic surface mapping algorithm), oracle version.

The steps follow the paper's overview of the method (Sec. 2.2 and the flow
chart there):
  1. collect the sources and images inside the auxiliary region (the near
     set S: 27 cells for the periodic box, Eq. 3; 9 cells x (2M+1) image
     layers for the dielectric slab, Eq. 4); with near_rule=1 only the
     images inside the auxiliary sphere itself, as Sec. 2.2 words it;
  2. evaluate the near potential Phi_B at the check points and fit the
     harmonic coefficients A by least squares, Eqs. (5)-(6);
  3. map the harmonic series to charges and dipoles on the sphere of radius
     R = lambda * (half box diagonal), integrated by a lattice (Fibonacci)
     rule;
  4. sum near set + sphere sources at the particles.
Outputs: energy E = 1/2 sum_i q_i Phi_i, potentials Phi_i, forces q_i E_i.
Units: Coulomb constant 1, eps_c = 1.

Readings where the paper is silent are documented next to the code:
check points on opposite box faces with value and normal-derivative
periodicity rows (3D); DtN rows on the two interfaces realised with a
spectral operator (2D); the constant coefficient A_0^0 fixed to zero.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import basis, geometry, native


class OracleInputError(ValueError):
    pass


def _check_neutral(q):
    q = np.asarray(q, dtype=np.float64)
    if abs(q.sum()) > 1e-12 * max(np.abs(q).sum(), 1e-300):
        raise OracleInputError("system is not charge neutral")


def _radius(L, lam):
    """R = lambda x half box diagonal; the diagonal as sqrt(Lx^2+Ly^2+Lz^2)
    summed left to right, so that the inside-the-sphere decision below is
    taken on exactly this R."""
    L = [float(v) for v in L]
    return lam * 0.5 * math.sqrt(L[0] * L[0] + L[1] * L[1] + L[2] * L[2])


def _cull_to_sphere(S, qS, self_idx, R):
    """The near set of Sec. 2.2 read literally: the images whose position
    lies strictly inside the auxiliary sphere |y| < R (box-centred).  The
    test is |y|^2 = (y_x^2 + y_y^2) + y_z^2 < R^2 in FP64 on the image
    positions as built (position + shift; z reflected, then shifted).  The
    candidates are the cell/layer stencil, which covers the sphere whenever
    R lies in the admissible range checked by the callers."""
    r2 = (S[:, 0] * S[:, 0] + S[:, 1] * S[:, 1]) + S[:, 2] * S[:, 2]
    keep = r2 < R * R
    if not np.all(keep[self_idx]):
        raise OracleInputError("a particle lies outside the auxiliary sphere")
    newidx = np.cumsum(keep) - 1
    return S[keep], qS[keep], newidx[self_idx]


@dataclass
class Result:
    energy: Optional[float]
    potential: np.ndarray      # at the requested targets
    field: np.ndarray          # E = -grad Phi at the targets
    force: np.ndarray          # q_t E_t
    A: np.ndarray              # harmonic coefficients (oracle basis)
    R: float
    Q: np.ndarray              # single-layer strengths on the sphere
    D: np.ndarray              # double-layer strengths on the sphere
    surface: tuple             # (points, normals, weights)
    rows: tuple                # (M, Y)
    check_data: dict


def _fit(M, Y):
    A, *_ = np.linalg.lstsq(M, Y, rcond=None)
    return A


def _surface_sources(A, R, p, F, rule, Fw):
    """Green's third identity on the sphere: for u harmonic inside,
    u(x) = (1/4pi) int [ d_n u(y) / |x-y| - u(y) n.(x-y)/|x-y|^3 ] dS_y,
    so u is the potential of charges Q_k = w_k d_n u(y_k) / 4pi and
    double-layer strengths D_k = w_k u(y_k) / 4pi."""
    y, nrm, w = geometry.surface_rule(F, R, rule, Fw)
    u = basis.values(y, R, p) @ A
    grad = np.einsum("kjc,kc->kj", basis.gradients(y, R, p), nrm)
    dn_u = grad @ A
    return y, nrm, w, w * dn_u / (4 * math.pi), w * u / (4 * math.pi)


def _final(x, q, S, qS, self_idx, y, nrm, Q, D, targets):
    tx = x[targets]
    skip = self_idx[targets]
    phi_n, E_n = native.charge_sums(tx, S, qS, skip=skip)
    phi_s, E_s = native.layer_sums(tx, y, nrm, Q, D)
    return phi_n + phi_s, E_n + E_s


def hsma3d(pos, q, box_lo, box_len, p, K, F, lam, Fw=0, surface_rule=0, targets=None, near_rule=0):
    """HSMA for the fully periodic box (tinfoil boundary at infinity).

    targets: optional index array of particles to evaluate (all if None);
    the energy is returned only when all particles are evaluated.
    near_rule: 0 = the 27 cells, 1 = the images inside the sphere."""
    L = np.asarray(box_len, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    _check_neutral(q)
    x = geometry.centre_and_wrap(pos, box_lo, L)
    R = _radius(L, lam)
    if not (0.5 * np.linalg.norm(L) < R < 1.5 * L.min()):
        raise OracleInputError("sphere radius outside (half diagonal, 1.5 min L)")
    nb = basis.nbasis(p)
    if 2 * K < nb:
        raise OracleInputError("fewer fitting rows than unknowns")

    # 1. near set
    S, qS, self_idx = geometry.images_3d(x, q, L)
    if near_rule == 1:
        S, qS, self_idx = _cull_to_sphere(S, qS, self_idx, R)
    elif near_rule != 0:
        raise OracleInputError("near_rule must be 0 or 1")

    # 2. least squares on periodicity rows at opposite face points
    xm, xp, axis = geometry.check_pairs_3d(L, K)
    phi_m, E_m = native.charge_sums(xm, S, qS)
    phi_p, E_p = native.charge_sums(xp, S, qS)
    k = np.arange(K)
    Ld = L[axis]
    gm = basis.gradients(xm, R, p)[k, :, axis]
    gp = basis.gradients(xp, R, p)[k, :, axis]
    M = np.vstack([basis.values(xp, R, p) - basis.values(xm, R, p), Ld[:, None] * (gp - gm)])
    # d/dx_d Phi_B = -E_d
    Y = np.concatenate([-(phi_p - phi_m), -Ld * (-E_p[k, axis] + E_m[k, axis])])
    A = _fit(M, Y)

    # 3. surface mapping
    y, nrm, w, Qk, Dk = _surface_sources(A, R, p, F, surface_rule, Fw)

    # 4. final sums
    tsel = np.arange(len(q)) if targets is None else np.asarray(targets)
    Phi, E = _final(x, q, S, qS, self_idx, y, nrm, Qk, Dk, tsel)
    energy = 0.5 * float(np.dot(q, Phi)) if targets is None else None
    return Result(energy, Phi, E, q[tsel][:, None] * E, A, R, Qk, Dk, (y, nrm, w), (M, Y),
                  dict(xm=xm, xp=xp, axis=axis, phi_m=phi_m, phi_p=phi_p, E_m=E_m, E_p=E_p))


def hsma2d(pos, q, box_lo, box_len, p, K, F, lam, M, gamma_up, gamma_low, nz,
           Fw=0, surface_rule=0, targets=None, near_rule=0):
    """HSMA for the slab periodic in x, y with dielectric interfaces at the
    two z faces of the box (mismatches gamma_up, gamma_low, |gamma| < 1).
    near_rule: 0 = 9 cells x (2M+1) layers, 1 = the images of those inside
    the sphere (M then only bounds the candidate layers)."""
    L = np.asarray(box_len, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    _check_neutral(q)
    x = geometry.centre_and_wrap(pos, box_lo, L, periodic=(True, True, False))
    h = 0.5 * L[2]
    if np.any(np.abs(x[:, 2]) >= h):
        raise OracleInputError("particle outside the slab")
    R = _radius(L, lam)
    if not (0.5 * np.linalg.norm(L) < R < min(1.5 * L[0], 1.5 * L[1], (M + 0.5) * L[2])):
        raise OracleInputError("sphere radius outside the admissible range")
    nb = basis.nbasis(p)

    # 1. near set with image layers
    S, qS, self_idx = geometry.images_2d(x, q, L, M, gamma_up, gamma_low)
    if near_rule == 1:
        S, qS, self_idx = _cull_to_sphere(S, qS, self_idx, R)
    elif near_rule != 0:
        raise OracleInputError("near_rule must be 0 or 1")

    # 2a. periodicity rows on the x and y faces
    xm, xp, axis = geometry.check_pairs_2d(L, K)
    phi_m, E_m = native.charge_sums(xm, S, qS)
    phi_p, E_p = native.charge_sums(xp, S, qS)
    k = np.arange(K)
    Ld = L[axis]
    gm = basis.gradients(xm, R, p)[k, :, axis]
    gp = basis.gradients(xp, R, p)[k, :, axis]
    M_per = np.vstack([basis.values(xp, R, p) - basis.values(xm, R, p), Ld[:, None] * (gp - gm)])
    Y_per = np.concatenate([-(phi_p - phi_m), -Ld * (-E_p[k, axis] + E_m[k, axis])])

    # 2b. dielectric (DtN) rows on the interfaces: exterior fields decay
    # like exp(-|G| dist), so continuity of Phi and of eps dPhi/dz give
    #   top:    (1+g_up) dPhi/dz + (1-g_up) T Phi = 0
    #   bottom: (1+g_low) dPhi/dz - (1-g_low) T Phi = 0
    # with T the spectral |G| operator on the interface grid; rows scaled by h.
    rows, rhs = [M_per], [Y_per]
    cd = dict(xm=xm, xp=xp, axis=axis, phi_m=phi_m, phi_p=phi_p, E_m=E_m, E_p=E_p)
    for top, gam, sgn in ((True, gamma_up, 1.0), (False, gamma_low, -1.0)):
        G = geometry.interface_grid(L, nz, top)
        phiB, EB = native.charge_sums(G, S, qS)
        b = basis.values(G, R, p)
        dzb = basis.gradients(G, R, p)[:, :, 2]
        rows.append(h * ((1 + gam) * dzb + sgn * (1 - gam) * geometry.spectral_dtn(b, L, nz)))
        rhs.append(-h * ((1 + gam) * (-EB[:, 2]) + sgn * (1 - gam) * geometry.spectral_dtn(phiB, L, nz)))
        cd["top" if top else "bottom"] = dict(points=G, phi=phiB, E=EB)
    Mrows = np.vstack(rows)
    Y = np.concatenate(rhs)
    if Mrows.shape[0] < nb:
        raise OracleInputError("fewer fitting rows than unknowns")
    A = _fit(Mrows, Y)

    # 3. surface mapping
    y, nrm, w, Qk, Dk = _surface_sources(A, R, p, F, surface_rule, Fw)

    # 4. final sums
    tsel = np.arange(len(q)) if targets is None else np.asarray(targets)
    Phi, E = _final(x, q, S, qS, self_idx, y, nrm, Qk, Dk, tsel)
    energy = 0.5 * float(np.dot(q, Phi)) if targets is None else None
    return Result(energy, Phi, E, q[tsel][:, None] * E, A, R, Qk, Dk, (y, nrm, w), (Mrows, Y), cd)


def far_series(A, R, p, pts):
    """The harmonic series sum_j A_j b_j(x) and its field -grad, evaluated
    directly (used to check the surface mapping)."""
    val = basis.values(pts, R, p) @ A
    grad = np.einsum("pjc,j->pc", basis.gradients(pts, R, p), A)
    return val, -grad


def run_workload(w, targets=None):
    """Evaluate a workloads.Workload with the oracle (positions from its seed)."""
    import workloads
    pos, q, lo, L = workloads.make_system(w)
    if w.geometry == 0:
        return hsma3d(pos, q, lo, L, w.p, w.K, w.F, w.lam, w.Fw, w.surface_rule, targets, w.near_rule)
    return hsma2d(pos, q, lo, L, w.p, w.K, w.F, w.lam, w.M, w.gamma_up, w.gamma_low, w.nz,
                  w.Fw, w.surface_rule, targets, w.near_rule)

"""Independent FP64 Ewald references (textbook forms, not from the paper).

ewald3d: fully periodic, conducting (tinfoil) boundary at infinity
  (Ewald 1921).  phi_i = real + reciprocal - self, E = -grad phi.
ewald2d: slab, periodic in x and y only (Parry 1975; Heyes, Barber &
  Clarke 1977), for an arbitrary neutral source set (e.g. dielectric image
  layers), with the reciprocal terms in an overflow-free erfcx form.

Both return potentials that exclude each target's own self interaction but
include all of its periodic (and image) copies.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc, erfcx, erf

SQPI = math.sqrt(math.pi)


def ewald3d(x, q, L, alpha=None, real_cut=None, tol=1e-17):
    """Potentials, fields and energy of a neutral periodic system."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    n = len(q)
    V = float(np.prod(L))
    if real_cut is None:
        real_cut = float(L.min())
    if alpha is None:
        alpha = 6.1 / real_cut                      # erfc(6.1) ~ 1e-18
    # real space: every image within real_cut of every target
    nsh = [int(math.ceil(real_cut / L[k])) + 1 for k in range(3)]
    phi = np.zeros(n)
    E = np.zeros((n, 3))
    for a in range(-nsh[0], nsh[0] + 1):
        for b in range(-nsh[1], nsh[1] + 1):
            for c in range(-nsh[2], nsh[2] + 1):
                sh = np.array([a, b, c]) * L
                d = x[:, None, :] - x[None, :, :] - sh
                r = np.sqrt(np.sum(d * d, axis=2))
                if a == 0 and b == 0 and c == 0:
                    np.fill_diagonal(r, np.inf)
                m = r < real_cut * 1.5
                rr = np.where(m, r, np.inf)
                er = erfc(alpha * rr) / rr
                phi += er @ q
                g = (er + 2 * alpha / SQPI * np.exp(-(alpha * rr) ** 2)) / (rr * rr)
                E += np.einsum("ij,ijk,j->ik", g, d, q)
    # reciprocal space over half the k lattice (k and -k pair up)
    kmax = 2 * alpha * math.sqrt(-math.log(tol))
    mmax = [int(math.ceil(kmax * L[k] / (2 * math.pi))) for k in range(3)]
    ms = np.array([(a, b, c) for a in range(-mmax[0], mmax[0] + 1)
                   for b in range(-mmax[1], mmax[1] + 1)
                   for c in range(-mmax[2], mmax[2] + 1)
                   if (a, b, c) > (0, 0, 0)], dtype=np.float64)
    kv = 2 * math.pi * ms / L
    k2 = np.sum(kv * kv, axis=1)
    keep = k2 <= kmax * kmax
    kv, k2 = kv[keep], k2[keep]
    coef = 2 * (4 * math.pi / V) * np.exp(-k2 / (4 * alpha * alpha)) / k2   # x2: half space
    for s in range(0, len(k2), 2048):
        ks = kv[s:s + 2048]
        ph = x @ ks.T                          # (n, nk)
        c, sn = np.cos(ph), np.sin(ph)
        Sc, Ss = q @ c, q @ sn                 # structure factor
        cs = coef[s:s + 2048]
        # sum_j q_j cos(k.(r_i - r_j)) = c_i Sc + s_i Ss
        phi += (c * Sc + sn * Ss) @ cs
        # sum_j q_j sin(k.(r_i - r_j)) = s_i Sc - c_i Ss
        E += ((sn * Sc - c * Ss) * cs) @ ks
    phi -= 2 * alpha / SQPI * q
    return phi, E, 0.5 * float(q @ phi)


def _slab_recip_term(G, z, alpha, s):
    """exp(s G z) erfc(G/(2 alpha) + s alpha z), evaluated without overflow."""
    xarg = G / (2 * alpha) + s * alpha * z
    pos = xarg >= 0
    out = np.empty(np.broadcast(G, z).shape)
    Gb, zb, xb = np.broadcast_arrays(G, z, xarg)
    out[pos] = np.exp(-(Gb[pos] / (2 * alpha)) ** 2 - (alpha * zb[pos]) ** 2) * erfcx(xb[pos])
    out[~pos] = np.exp(s * Gb[~pos] * zb[~pos]) * erfc(xb[~pos])
    return out


def ewald2d(tx, sx, sq, Lxy, self_idx=None, alpha=None, tol=1e-17, inplane_cut=None):
    """Potential and field at targets tx from a neutral source set (sx, sq)
    periodic in x and y with periods Lxy = (Lx, Ly).

    self_idx[t] marks the source that is target t itself (its self
    interaction is removed); sources may extend arbitrarily far in z."""
    tx = np.asarray(tx, dtype=np.float64)
    sx = np.asarray(sx, dtype=np.float64)
    sq = np.asarray(sq, dtype=np.float64)
    Lx, Ly = float(Lxy[0]), float(Lxy[1])
    A = Lx * Ly
    nt = len(tx)
    if inplane_cut is None:
        inplane_cut = min(Lx, Ly)
    if alpha is None:
        alpha = 6.1 / inplane_cut
    phi = np.zeros(nt)
    E = np.zeros((nt, 3))
    ns = [int(math.ceil(inplane_cut / Lx)) + 1, int(math.ceil(inplane_cut / Ly)) + 1]
    is_self = np.zeros((nt, len(sq)), dtype=bool)
    if self_idx is not None:
        is_self[np.arange(nt), np.asarray(self_idx)] = True
    # real space (only sources within reach of erfc contribute)
    for a in range(-ns[0], ns[0] + 1):
        for b in range(-ns[1], ns[1] + 1):
            sh = np.array([a * Lx, b * Ly, 0.0])
            d = tx[:, None, :] - sx[None, :, :] - sh
            r = np.sqrt(np.sum(d * d, axis=2))
            if a == 0 and b == 0:
                r = np.where(is_self, np.inf, r)
            rr = np.where(r < 1.5 * inplane_cut, r, np.inf)
            er = erfc(alpha * rr) / rr
            phi += er @ sq
            g = (er + 2 * alpha / SQPI * np.exp(-(alpha * rr) ** 2)) / (rr * rr)
            E += np.einsum("ij,ijk,j->ik", g, d, sq)
    # reciprocal, G != 0 (half plane, doubled)
    Gmax = 2 * alpha * math.sqrt(-math.log(tol))
    mx = int(math.ceil(Gmax * Lx / (2 * math.pi)))
    my = int(math.ceil(Gmax * Ly / (2 * math.pi)))
    dxy = tx[:, None, :2] - sx[None, :, :2]
    zz = tx[:, None, 2] - sx[None, :, 2]
    for a in range(-mx, mx + 1):
        for b in range(-my, my + 1):
            if (a, b) <= (0, 0):
                continue
            gv = np.array([2 * math.pi * a / Lx, 2 * math.pi * b / Ly])
            G = math.hypot(gv[0], gv[1])
            if G > Gmax:
                continue
            cosg = np.cos(dxy @ gv)
            sing = np.sin(dxy @ gv)
            tp = _slab_recip_term(G, zz, alpha, 1.0)
            tm = _slab_recip_term(G, zz, alpha, -1.0)
            pref = 2 * math.pi / A          # pi/A x2 for the half plane
            phi += pref / G * ((cosg * (tp + tm)) @ sq)
            fxy = pref / G * ((sing * (tp + tm)) @ sq)
            E[:, 0] += fxy * gv[0]
            E[:, 1] += fxy * gv[1]
            E[:, 2] += -pref * ((cosg * (tp - tm)) @ sq)
    # G = 0
    phi += -(2 * math.pi / A) * ((zz * erf(alpha * zz) + np.exp(-(alpha * zz) ** 2) / (alpha * SQPI)) @ sq)
    E[:, 2] += (2 * math.pi / A) * (erf(alpha * zz) @ sq)
    if self_idx is not None:
        phi -= 2 * alpha / SQPI * sq[np.asarray(self_idx)]
    return phi, E


def slab_reference(x, q, L, gamma_up, gamma_low, M_ref, targets=None):
    """Exact slab electrostatics with image layers up to order M_ref (enough
    that |gamma|^M_ref is negligible), via ewald2d.  x: centred positions."""
    from . import geometry
    S, qS, self_idx = geometry.images_2d(x, q, L, M_ref, gamma_up, gamma_low, inplane=0)
    tsel = np.arange(len(q)) if targets is None else np.asarray(targets)
    phi, E = ewald2d(x[tsel], S, qS, L[:2], self_idx=self_idx[tsel])
    energy = 0.5 * float(q @ phi) if targets is None else None
    return phi, E, energy

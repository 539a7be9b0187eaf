"""Pins of the FP64 oracle against things other than itself: closed forms,
brute force, independent Ewald sums, invariants, and planted mistakes."""
import json
import math
import os

import numpy as np
import pytest
from scipy.special import sph_harm_y

import workloads
from oracle import basis, ewald, geometry, hsma, native

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CONST = json.load(open(os.path.join(GOLD, "reference_constants.json")))
PAPER = json.load(open(os.path.join(GOLD, "paper_parameters.json")))
NACL_M = CONST["nacl_madelung"]["value"]


def nacl_cell(a=5.0, offset=(0.37, 0.61, 0.23)):
    base = np.array([[0, 0, 0], [1, 1, 0], [1, 0, 1], [0, 1, 1]], float) * a
    x = np.vstack([base, base + np.array([a, 0, 0])]) + np.array(offset)
    q = np.array([1.0] * 4 + [-1.0] * 4)
    return x, q, np.zeros(3), np.array([2 * a] * 3)


# ------------------------------------------------------------ pair sums
def test_charge_sums_match_brute_force():
    rng = np.random.default_rng(1)
    t = rng.random((7, 3)) * 3
    s = rng.random((11, 3)) * 3
    qs = rng.standard_normal(11)
    skip = np.array([-1, 2, -1, 0, 10, -1, 5])
    phi, E = native.charge_sums(t, s, qs, skip)
    for i in range(7):
        p, e = 0.0, np.zeros(3)
        for j in range(11):
            if j == skip[i]:
                continue
            d = t[i] - s[j]
            r = math.sqrt(d @ d)
            p += qs[j] / r
            e += qs[j] * d / r ** 3
        assert abs(phi[i] - p) < 1e-13 * max(1, abs(p))
        assert np.allclose(E[i], e, rtol=1e-13, atol=1e-13)


def test_layer_sums_field_is_minus_gradient():
    rng = np.random.default_rng(2)
    y = rng.standard_normal((9, 3)) * 5
    n = rng.standard_normal((9, 3))
    n /= np.linalg.norm(n, axis=1)[:, None]
    Q, D = rng.standard_normal(9), rng.standard_normal(9)
    x = rng.random((4, 3))
    phi, E = native.layer_sums(x, y, n, Q, D)
    h = 1e-5
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fp, _ = native.layer_sums(x + e, y, n, Q, D)
        fm, _ = native.layer_sums(x - e, y, n, Q, D)
        assert np.allclose(-(fp - fm) / (2 * h), E[:, k], rtol=1e-7, atol=1e-8)
    # a dipole of strength D along n is the limit of two charges +-D/eps
    # placed at y -+ eps n/2 (moment -D n): check the potential.
    eps = 1e-4
    src = np.vstack([y - 0.5 * eps * n, y + 0.5 * eps * n])
    qq = np.concatenate([D / eps, -D / eps])
    pd, _ = native.charge_sums(x, src, qq)
    p0, _ = native.layer_sums(x, y, n, np.zeros(9), D)
    assert np.allclose(p0, pd, rtol=1e-6, atol=1e-8)


# ------------------------------------------------------------ Ewald 3D
def test_ewald3d_nacl_madelung():
    x, q, lo, L = nacl_cell()
    xc = geometry.centre_and_wrap(x, lo, L)
    phi, E, en = ewald.ewald3d(xc, q, L)
    a = L[0] / 2
    assert abs(en - (-4 * NACL_M / a)) < 1e-13
    assert np.abs(E).max() < 1e-13
    assert np.allclose(phi * q, -NACL_M / a, atol=1e-13)


def test_ewald3d_alpha_independent_and_newton():
    pos, q, lo, L = workloads.small_system(30, (6.0, 7.0, 8.0), 3)
    x = geometry.centre_and_wrap(pos, lo, L)
    p1, E1, e1 = ewald.ewald3d(x, q, L)
    p2, E2, e2 = ewald.ewald3d(x, q, L, alpha=1.3, real_cut=4.0)
    assert abs(e1 - e2) < 1e-12 * abs(e1)
    assert np.abs(E1 - E2).max() < 1e-11 * np.abs(E1).max()
    assert np.abs((q[:, None] * E1).sum(0)).max() < 1e-12 * np.abs(E1).max()


# ------------------------------------------------------------ Ewald 2D
def test_ewald2d_square_lattice_madelung():
    a = 1.0
    x = np.array([[0, 0, 0], [1, 1, 0], [1, 0, 0], [0, 1, 0]], float) * a + [0.3, 0.2, 0.0]
    q = np.array([1, 1, -1, -1.0])
    phi, E = ewald.ewald2d(x, x, q, (2 * a, 2 * a), self_idx=np.arange(4), alpha=1.7)
    M = CONST["square_checkerboard_madelung"]["value"]
    assert np.allclose(q * phi, -M / a, atol=1e-12)
    assert np.abs(E).max() < 1e-12


def test_ewald2d_matches_ewald3d_with_vacuum_and_dipole_correction():
    # Yeh-Berkowitz: a slab in a tall periodic box plus 2 pi M_z^2 / V
    rng = np.random.default_rng(0)
    L = np.array([4.0, 5.0, 3.0])
    x = rng.random((10, 3)) * L - L / 2
    q = np.array([1.0, -1.0] * 5)
    p2, E2 = ewald.ewald2d(x, x, q, L[:2], self_idx=np.arange(10))
    p2b, E2b = ewald.ewald2d(x, x, q, L[:2], self_idx=np.arange(10), alpha=3.0)
    assert np.abs(p2 - p2b).max() < 1e-12
    L3 = np.array([4.0, 5.0, 60.0])
    p3, E3, e3 = ewald.ewald3d(x, q, L3, real_cut=4.0)
    Mz = q @ x[:, 2]
    V = np.prod(L3)
    assert abs(e3 + 2 * math.pi / V * Mz ** 2 - 0.5 * q @ p2) < 1e-12
    assert np.abs(E3[:, 2] - 4 * math.pi / V * Mz - E2[:, 2]).max() < 1e-12
    assert np.abs(E3[:, :2] - E2[:, :2]).max() < 1e-12


# ------------------------------------------------------------ basis
@pytest.mark.parametrize("p", [1, 4, 12])
def test_basis_is_harmonic_with_right_dimension(p):
    for n, C in enumerate(basis.harmonic_basis(p), 1):
        assert C.shape == (len(basis.monomials(n)), 2 * n + 1)
        lap = basis.laplacian_matrix(n)
        if lap.shape[0]:
            assert np.abs(lap @ C).max() < 1e-13 * np.abs(lap).sum(1).max() * np.abs(C).max()
    assert basis.nbasis(p) == (p + 1) ** 2 - 1


def test_basis_spans_library_spherical_harmonics():
    p, R = 8, 2.5
    rng = np.random.default_rng(4)
    pts = rng.standard_normal((400, 3))
    pts *= (rng.random(400) * 1.2 * R / np.linalg.norm(pts, axis=1))[:, None]
    B = basis.values(pts, R, p)
    r = np.linalg.norm(pts, axis=1)
    th = np.arccos(pts[:, 2] / r)
    ph = np.arctan2(pts[:, 1], pts[:, 0])
    for n in range(1, p + 1):
        for m in range(0, n + 1):
            Y = sph_harm_y(n, m, th, ph) * (r / R) ** n
            for part in (Y.real, Y.imag):
                if np.abs(part).max() < 1e-12:
                    continue
                coef, *_ = np.linalg.lstsq(B, part, rcond=None)
                assert np.abs(B @ coef - part).max() < 1e-10 * np.abs(part).max()


def test_basis_orthonormal_on_sphere_and_gradients():
    p = 6
    ct, wt = np.polynomial.legendre.leggauss(20)
    ph = 2 * np.pi * np.arange(41) / 41
    st = np.sqrt(1 - ct ** 2)
    pts = np.stack([np.outer(st, np.cos(ph)).ravel(), np.outer(st, np.sin(ph)).ravel(), np.repeat(ct, 41)], 1)
    w = np.repeat(wt, 41) * 2 * np.pi / 41
    B = basis.values(pts, 1.0, p)
    G = B.T @ (w[:, None] * B)
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-12
    rng = np.random.default_rng(5)
    x = rng.standard_normal((6, 3))
    g = basis.gradients(x, 1.7, p)
    h = 1e-6
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        fd = (basis.values(x + e, 1.7, p) - basis.values(x - e, 1.7, p)) / (2 * h)
        assert np.allclose(fd, g[:, :, k], rtol=1e-6, atol=1e-7)


# ------------------------------------------------------------ quadrature
@pytest.mark.parametrize("rule,F", [(0, 800), (1, 800), (0, 89)])
def test_surface_rule_integrates(rule, F):
    R = 3.0
    y, n, w = geometry.surface_rule(F, R, rule)
    assert np.allclose(np.linalg.norm(n, axis=1), 1.0)
    assert np.allclose(y, R * n)
    tol = {800: 1e-9, 89: 1e-3}[F] if rule == 0 else 1e-12
    assert abs(w.sum() - 4 * math.pi * R * R) < tol * 4 * math.pi * R * R
    assert abs(w @ y[:, 0] ** 2 - 4 * math.pi * R ** 4 / 3) < tol * R ** 4 * 10
    # products of two degree-p harmonics have degree 2p; 89 points resolve
    # only p = 2 (the paper's F = 89 cannot integrate P = 10 products)
    p = 2 if F == 89 else 8
    B = basis.values(y, R, p)
    G = B.T @ (w[:, None] * B) / R ** 2
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-6


def test_fibonacci_generator_and_zaremba():
    assert geometry.lattice_generator(89) == 55
    assert geometry.lattice_generator(PAPER["hsma3d_recommended"]["F"]) == PAPER["hsma3d_recommended"]["F_w"]
    for F in (200, 512, 800, 1152):
        g = geometry.lattice_generator(F)
        z = geometry.zaremba_index(F, g)
        assert all(geometry.zaremba_index(F, h) <= z for h in range(1, F // 2 + 1))


def test_green_mapping_reproduces_series():
    """The surface charges/dipoles reproduce the harmonic series inside the
    sphere (Green's third identity), converging with F."""
    rng = np.random.default_rng(6)
    p, R = 8, 10.0
    A = rng.standard_normal(basis.nbasis(p)) * np.repeat(0.7 ** np.arange(1, p + 1), 2 * np.arange(1, p + 1) + 1)
    x = rng.uniform(-1, 1, (50, 3)) * R / (1.5 * math.sqrt(3))
    v, e = hsma.far_series(A, R, p, x)
    errs = []
    for F in (200, 800, 1152):
        y, nrm, w, Q, D = hsma._surface_sources(A, R, p, F, 1, 0)
        pv, pe = native.layer_sums(x, y, nrm, Q, D)
        errs.append(np.abs(pv - v).max() / np.abs(v).max())
        assert np.abs(pe - e).max() / np.abs(e).max() < 100 * errs[-1] + 1e-9
    assert errs[-1] < 1e-8 and errs[0] > errs[-1]


# ------------------------------------------------------------ images
def test_image_layers_follow_reflection_recursion():
    rng = np.random.default_rng(7)
    L = np.array([3.0, 4.0, 2.0])
    h = 1.0
    x = rng.uniform(-1, 1, (5, 3)) * [1.5, 2.0, 0.9]
    q = rng.standard_normal(5)
    gu, gl, M = 0.6, -0.3, 5
    S, qS, self_idx = geometry.images_2d(x, q, L, M, gu, gl, inplane=0)
    n = 5
    layers = {0: (x, q)}
    # layout per in-plane shift: sources, then (up_l, low_l) for l = 1..M
    for l in range(1, M + 1):
        up = (S[(2 * l - 1) * n:(2 * l) * n], qS[(2 * l - 1) * n:(2 * l) * n])
        lo = (S[(2 * l) * n:(2 * l + 1) * n], qS[(2 * l) * n:(2 * l + 1) * n])
        layers[("u", l)] = up
        layers[("d", l)] = lo
    def refl_top(z):
        return 2 * h - z
    def refl_bot(z):
        return -2 * h - z
    # U_1 = g_up Refl_top(sources), D_1 = g_low Refl_bot(sources)
    assert np.allclose(layers[("u", 1)][0][:, 2], refl_top(x[:, 2]))
    assert np.allclose(layers[("u", 1)][1], gu * q)
    assert np.allclose(layers[("d", 1)][0][:, 2], refl_bot(x[:, 2]))
    assert np.allclose(layers[("d", 1)][1], gl * q)
    for l in range(1, M):
        U, Dn = layers[("u", l + 1)], layers[("d", l + 1)]
        assert np.allclose(U[0][:, 2], refl_top(layers[("d", l)][0][:, 2]))
        assert np.allclose(U[1], gu * layers[("d", l)][1])
        assert np.allclose(Dn[0][:, 2], refl_bot(layers[("u", l)][0][:, 2]))
        assert np.allclose(Dn[1], gl * layers[("u", l)][1])
        assert np.allclose(U[0][:, :2], x[:, :2]) and np.allclose(Dn[0][:, :2], x[:, :2])
    assert np.all(S[self_idx] == x)


def test_single_interface_image_energy_and_force():
    """gamma_low = 0: one interface.  A charge at distance d below the top
    interface sees its image only: energy gamma q^2/(4d), force
    gamma q^2/(4d^2) away from the interface."""
    gam, qv, d, h = 0.7, 1.5, 0.3, 1.0
    x = np.array([[0.0, 0.0, h - d]])
    S, qS, self_idx = geometry.images_2d(x, np.array([qv]), np.array([50.0, 50.0, 2 * h]), 6, gam, 0.0, inplane=0)
    phi, E = native.charge_sums(x, S, qS, skip=self_idx)
    assert abs(0.5 * qv * phi[0] - gam * qv * qv / (4 * d)) < 1e-14
    assert abs(qv * E[0, 2] + gam * qv * qv / (4 * d * d)) < 1e-13


# ------------------------------------------------------------ HSMA3D
def test_hsma3d_nacl_within_method_error():
    x, q, lo, L = nacl_cell()
    a = L[0] / 2
    r6 = hsma.hsma3d(x, q, lo, L, 6, 100, 200, 1.5)
    assert abs(r6.energy / (-4 * NACL_M / a) - 1) < 1e-4
    assert np.abs(r6.force).max() < 1e-4
    r12 = hsma.hsma3d(x, q, lo, L, 12, 800, 1152, 1.5, surface_rule=1)
    assert abs(r12.energy / (-4 * NACL_M / a) - 1) < 5e-6


def test_hsma3d_config1_against_ewald():
    pos, q, lo, L = workloads.make_system(workloads.C1)
    xc = geometry.centre_and_wrap(pos, lo, L)
    _, E, en = ewald.ewald3d(xc, q, L)
    Fref = q[:, None] * E
    for p, K, F, tol_e, tol_f in ((6, 100, 200, 5e-5, 2e-4), (10, 400, 800, 1e-6, 1e-5)):
        r = hsma.hsma3d(pos, q, lo, L, p, K, F, 1.5)
        assert abs(r.energy - en) < tol_e * abs(en)
        assert np.sqrt(((r.force - Fref) ** 2).sum() / (Fref ** 2).sum()) < tol_f
        # potentials agree modulo the undetermined constant
        pd = r.potential - geometry.centre_and_wrap(pos, lo, L)[:, 0] * 0
        phi_ref = _ewald_phi(xc, q, L)
        dp = (r.potential - r.potential.mean()) - (phi_ref - phi_ref.mean())
        assert np.abs(dp).max() < 20 * tol_f * np.abs(phi_ref).max()


def _ewald_phi(x, q, L):
    return ewald.ewald3d(x, q, L)[0]


def test_hsma3d_scaling_permutation_and_lsq_optimality():
    pos, q, lo, L = workloads.small_system(40, (8.0, 8.0, 8.0), 11)
    r = hsma.hsma3d(pos, q, lo, L, 6, 100, 200, 1.5)
    s = 2.5
    rs = hsma.hsma3d(pos * s, q, lo * s, L * s, 6, 100, 200, 1.5)
    assert abs(rs.energy - r.energy / s) < 1e-12 * abs(r.energy)
    assert np.abs(rs.force - r.force / s ** 2).max() < 1e-11 * np.abs(r.force).max()
    perm = np.random.default_rng(3).permutation(40)
    rp = hsma.hsma3d(pos[perm], q[perm], lo, L, 6, 100, 200, 1.5)
    assert abs(rp.energy - r.energy) < 1e-12 * abs(r.energy)
    assert np.abs(rp.force - r.force[perm]).max() < 1e-11 * np.abs(r.force).max()
    M, Y = r.rows
    g = M.T @ (M @ r.A - Y)
    assert np.abs(g).max() < 1e-10 * np.abs(M.T @ Y).max()
    # net force vanishes within method error
    assert np.abs(r.force.sum(0)).max() < 1e-4 * np.sqrt((r.force ** 2).sum())
    # translation: the physics is invariant, HSMA within its error
    shift = np.array([1.3, -0.7, 2.2])
    rt = hsma.hsma3d(pos + shift, q, lo, L, 6, 100, 200, 1.5)
    assert abs(rt.energy - r.energy) < 1e-4 * abs(r.energy)


def test_hsma3d_force_is_minus_energy_gradient():
    """Finite differences of the HSMA energy against the reported forces
    F_i = q_i E_i, within the method error (the fit is redone at every
    displaced configuration, so agreement is at the method-error level, not
    to rounding)."""
    pos, q, lo, L = workloads.make_system(workloads.C1)
    p, K, F = 8, 162, 512
    r = hsma.hsma3d(pos, q, lo, L, p, K, F, 1.5)
    scale = np.abs(r.force).max()
    h = 1e-4
    for i in (3, 41, 77):
        for k in range(3):
            pp = pos.copy()
            pp[i, k] += h
            ep = hsma.hsma3d(pp, q, lo, L, p, K, F, 1.5).energy
            pp[i, k] -= 2 * h
            em = hsma.hsma3d(pp, q, lo, L, p, K, F, 1.5).energy
            fd = -(ep - em) / (2 * h)
            assert abs(fd - r.force[i, k]) < 1e-5 * scale, (i, k, fd, r.force[i, k])  # measured 1.1e-6


def test_hsma3d_rejects_bad_input():
    pos, q, lo, L = workloads.small_system(10, (5.0, 5.0, 5.0), 1)
    with pytest.raises(hsma.OracleInputError):
        hsma.hsma3d(pos, q + 0.1, lo, L, 4, 50, 200, 1.5)
    with pytest.raises(hsma.OracleInputError):
        hsma.hsma3d(pos, q, lo, L, 4, 50, 200, 2.0)   # sphere reaches far cells
    with pytest.raises(hsma.OracleInputError):
        hsma.hsma3d(pos, q, lo, L, 6, 10, 200, 1.5)   # 20 rows < 48 unknowns


def test_hsma3d_sphere_near_set_against_ewald():
    """near_rule=1 (only the images inside the auxiliary sphere, Sec. 2.2):
    an exact split as well, so the result converges to Ewald as p grows;
    its far field starts at R instead of 1.5 L, so it needs a higher p than
    the 27-cell set for the same error."""
    pos, q, lo, L = workloads.make_system(workloads.C1)
    xc = geometry.centre_and_wrap(pos, lo, L)
    _, E, en = ewald.ewald3d(xc, q, L)
    Fref = q[:, None] * E
    errs = []
    for p, K, F, tol_e, tol_f in ((6, 100, 200, 3e-3, 5e-3), (12, 800, 1152, 3e-5, 5e-5)):
        r = hsma.hsma3d(pos, q, lo, L, p, K, F, 1.5, near_rule=1)
        de = abs(r.energy - en) / abs(en)
        df = np.sqrt(((r.force - Fref) ** 2).sum() / (Fref ** 2).sum())
        assert de < tol_e and df < tol_f
        errs.append(df)
    assert errs[1] < errs[0] / 20


def test_sphere_near_set_is_every_image_inside():
    """The culled stencil holds exactly the images inside the sphere: the
    same set comes out of a 7x7x7-cell (slab: 7x7 cells, M+4 layers)
    candidate set, so no image inside the sphere lies beyond the stencil."""
    pos, q, lo, L = workloads.small_system(30, (6.0, 7.0, 6.5), 21)
    x = geometry.centre_and_wrap(pos, lo, L)
    R = hsma._radius(L, 1.5)
    S, qS, si = hsma._cull_to_sphere(*geometry.images_3d(x, q, L), R)
    ks = np.array([(a, b, c) for a in range(-3, 4) for b in range(-3, 4) for c in range(-3, 4)], dtype=np.float64)
    W = (x[None, :, :] + (ks * L)[:, None, :]).reshape(-1, 3)
    Win = W[np.linalg.norm(W, axis=1) < R]
    assert len(Win) == len(S) and 9 * len(q) < len(S) < 27 * len(q)
    key = lambda A: A[np.lexsort(A.T)]
    assert np.abs(key(Win) - key(S)).max() < 1e-12
    assert np.all(np.linalg.norm(S[si] - x, axis=1) == 0)
    # slab
    pos, q, lo, L = workloads.small_system(20, (20.0, 20.0, 10.0), 5, geometry=1)
    x = geometry.centre_and_wrap(pos, lo, L, periodic=(True, True, False))
    R = hsma._radius(L, 1.6)
    S, qS, si = hsma._cull_to_sphere(*geometry.images_2d(x, q, L, 6, -0.5, 0.3), R)
    W, qW, _ = geometry.images_2d(x, q, L, 10, -0.5, 0.3, inplane=3)
    inside = np.linalg.norm(W, axis=1) < R
    assert inside.sum() == len(S)
    assert abs(qW[inside].sum() - qS.sum()) < 1e-12 and abs((qW[inside] ** 2).sum() - (qS ** 2).sum()) < 1e-12


# ------------------------------------------------------------ HSMA2D
@pytest.mark.parametrize("gam,Mref,nz", [(0.0, 0, 160), (-0.94, 560, 160), (0.5, 50, 80)])
def test_hsma2d_against_ewald2d_image_sum(gam, Mref, nz):
    """End-to-end pin of the 2D reading.  An ion sits 0.57 from a wall in
    this system: the interface grid must resolve its peak (nz = 160 gives
    ~4e-6; nz = 80 aliases to ~5e-4 at gamma = 0)."""
    pos, q, lo, L = workloads.small_system(12, (40.0, 40.0, 20.0), 7, geometry=1)
    x = geometry.centre_and_wrap(pos, lo, L, periodic=(True, True, False))
    _, E, en = ewald.slab_reference(x, q, L, gam, gam, Mref)
    Fref = q[:, None] * E
    r = hsma.hsma2d(pos, q, lo, L, 10, 400, 800, 1.6, 10, gam, gam, nz)
    tol = 2e-5 if nz == 160 else 1e-3
    assert abs(r.energy - en) < tol * abs(en)
    assert np.sqrt(((r.force - Fref) ** 2).sum() / (Fref ** 2).sum()) < tol
    # in-plane net force vanishes
    assert np.abs(r.force[:, :2].sum(0)).max() < 20 * tol * np.sqrt((r.force ** 2).sum())


@pytest.mark.parametrize("gam,Mref,tol", [(-0.94, 560, 5e-5), (0.5, 50, 3e-5)])
def test_hsma2d_sphere_near_set_against_image_sum(gam, Mref, tol):
    """near_rule=1 for the slab: image layers beyond the sphere move into
    the fitted far field; p = 12 reaches the image-sum reference (ions kept
    2 from the walls so that nz = 40 resolves them)."""
    pos, q, lo, L = workloads.small_system(12, (20.0, 20.0, 10.0), 7, geometry=1, z_margin=2.0)
    x = geometry.centre_and_wrap(pos, lo, L, periodic=(True, True, False))
    _, E, en = ewald.slab_reference(x, q, L, gam, gam, Mref)
    Fref = q[:, None] * E
    r = hsma.hsma2d(pos, q, lo, L, 12, 800, 1152, 1.6, 10, gam, gam, 40, near_rule=1)
    assert abs(r.energy - en) < tol * abs(en)
    assert np.sqrt(((r.force - Fref) ** 2).sum() / (Fref ** 2).sum()) < tol


def test_hsma2d_mirror_symmetry():
    pos, q, lo, L = workloads.small_system(10, (20.0, 20.0, 10.0), 9, geometry=1)
    r = hsma.hsma2d(pos, q, lo, L, 6, 100, 200, 1.6, 6, -0.5, -0.5, 40, surface_rule=1)
    pm = pos.copy()
    pm[:, 2] = L[2] - pos[:, 2]
    rm = hsma.hsma2d(pm, q, lo, L, 6, 100, 200, 1.6, 6, -0.5, -0.5, 40, surface_rule=1)
    assert abs(rm.energy - r.energy) < 1e-3 * abs(r.energy)
    Fm = rm.force.copy()
    Fm[:, 2] *= -1
    assert np.abs(Fm - r.force).max() < 1e-3 * np.abs(r.force).max()


def test_hsma2d_in_plane_translation():
    """Shifting every ion in x and y (the slab is periodic there) leaves the
    energy unchanged and moves the forces with the ions, within the method
    error."""
    pos, q, lo, L = workloads.small_system(10, (20.0, 20.0, 10.0), 9, geometry=1)
    args = (6, 100, 200, 1.6, 6, -0.5, -0.5, 40)
    r = hsma.hsma2d(pos, q, lo, L, *args, surface_rule=1)
    shifted = pos + np.array([7.3, -12.1, 0.0])
    rs = hsma.hsma2d(shifted, q, lo, L, *args, surface_rule=1)
    assert abs(rs.energy - r.energy) < 1e-3 * abs(r.energy)
    assert np.abs(rs.force - r.force).max() < 1e-3 * np.abs(r.force).max()


def test_hsma2d_rejects_particle_outside_slab():
    pos, q, lo, L = workloads.small_system(10, (20.0, 20.0, 10.0), 9, geometry=1)
    pos[0, 2] = 10.5
    with pytest.raises(hsma.OracleInputError):
        hsma.hsma2d(pos, q, lo, L, 4, 50, 200, 1.6, 4, 0.1, 0.1, 20)


# ------------------------------------------------------------ planted mistakes
def test_planted_mistakes_are_caught(monkeypatch):
    """Each plausible slip in the oracle breaks a pin above."""
    pos, q, lo, L = workloads.make_system(workloads.C1)
    xc = geometry.centre_and_wrap(pos, lo, L)
    _, E, _ = ewald.ewald3d(xc, q, L)
    Fref = q[:, None] * E

    def err():
        r = hsma.hsma3d(pos, q, lo, L, 6, 100, 200, 1.5)
        return np.sqrt(((r.force - Fref) ** 2).sum() / (Fref ** 2).sum())

    base = err()
    assert base < 2e-4
    # (1) wrong sign of the double layer
    orig = hsma._surface_sources

    def flipped(*args):
        y, n, w, Q, D = orig(*args)
        return y, n, w, Q, -D
    monkeypatch.setattr(hsma, "_surface_sources", flipped)
    assert err() > 30 * base
    monkeypatch.setattr(hsma, "_surface_sources", orig)
    # (2) a dropped single-layer term
    def no_charge(*args):
        y, n, w, Q, D = orig(*args)
        return y, n, w, 0 * Q, D
    monkeypatch.setattr(hsma, "_surface_sources", no_charge)
    assert err() > 30 * base
    monkeypatch.setattr(hsma, "_surface_sources", orig)
    # (3) the paper's printed image exponents fail the single-interface pin
    orig_s = geometry.image_strengths
    monkeypatch.setattr(geometry, "image_strengths",
                        lambda l, gu, gl: (gl ** ((l + 1) // 2) * gu ** (l // 2), gu ** ((l + 1) // 2) * gl ** (l // 2)))
    with pytest.raises(AssertionError):
        test_single_interface_image_energy_and_force()
    monkeypatch.setattr(geometry, "image_strengths", orig_s)
    # (4) x+ placed on the wrong face: the fit no longer enforces periodicity
    orig_c = geometry.check_pairs_3d

    def bad_pairs(L, K):
        xm, xp, ax = orig_c(L, K)
        xp = xm.copy()
        xp[np.arange(K), (ax + 1) % 3] += 0.5 * np.asarray(L)[(ax + 1) % 3]
        return xm, xp, ax
    monkeypatch.setattr(geometry, "check_pairs_3d", bad_pairs)
    assert err() > 30 * base
    monkeypatch.setattr(geometry, "check_pairs_3d", orig_c)

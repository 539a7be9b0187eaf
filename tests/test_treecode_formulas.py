"""CPU checks of the expansion formulas the treecode kernels use (near rule
2): the solid-harmonic recursions, the addition theorem, the derivative
relations behind the field, the moment shift, and the mirror rule for the
slab's image layers.  Independent re-statements in numpy (the kernels are
tested end to end against the oracle's exact sums on the GPU)."""
import numpy as np
import pytest


def regular(P, v):
    """U_n^m(v), m >= 0: U_0^0 = 1, U_m^m = (x + iy)/(2m) U_{m-1}^{m-1},
    U_n^m = ((2n-1) z U_{n-1}^m - r^2 U_{n-2}^m) / ((n+m)(n-m))."""
    x, y, z = v
    r2 = x * x + y * y + z * z
    U = np.zeros((P + 1, P + 1), complex)
    U[0, 0] = 1.0
    for n in range(1, P + 1):
        U[n, n] = (x + 1j * y) / (2 * n) * U[n - 1, n - 1]
        for m in range(n):
            U[n, m] = ((2 * n - 1) * z * U[n - 1, m] - (r2 * U[n - 2, m] if n >= 2 else 0)) / ((n + m) * (n - m))
    return U


def irregular(P, v):
    """T_n^m(v), m >= 0: T_0^0 = 1/r, T_m^m = (2m-1)(x + iy)/r^2 T_{m-1}^{m-1},
    T_n^m = ((2n-1) z T_{n-1}^m - ((n-1)^2 - m^2) T_{n-2}^m) / r^2."""
    x, y, z = v
    r2 = x * x + y * y + z * z
    T = np.zeros((P + 1, P + 1), complex)
    T[0, 0] = 1.0 / np.sqrt(r2)
    for n in range(1, P + 1):
        T[n, n] = (2 * n - 1) * (x + 1j * y) / r2 * T[n - 1, n - 1]
        for m in range(n):
            T[n, m] = ((2 * n - 1) * z * T[n - 1, m] - (((n - 1) ** 2 - m * m) * T[n - 2, m] if n >= 2 else 0)) / r2
    return T


def at(A, n, m):
    """X_n^m for any |m| <= n from the m >= 0 table: X_n^{-m} = (-1)^m conj(X_n^m)."""
    if abs(m) > n:
        return 0.0
    return A[n, m] if m >= 0 else (-1) ** m * np.conj(A[n, -m])


def expansion(P, M, X):
    """Potential and field of moments M at X, as the kernel folds them
    (column 0 alone, the conjugate columns counted twice)."""
    T = irregular(P + 1, X)
    phi0 = phi1 = dz0 = dz1 = 0.0
    W = 0.0
    for n in range(P + 2):
        for m in range(0, n + 1):
            t = T[n, m]
            if n <= P:
                v = (np.conj(M[n, m]) * t).real
                phi0, phi1 = (phi0 + v, phi1) if m == 0 else (phi0, phi1 + v)
            if n >= 1 and n - 1 >= m:
                v = (np.conj(M[n - 1, m]) * t).real
                dz0, dz1 = (dz0 + v, dz1) if m == 0 else (dz0, dz1 + v)
            if m >= 1:
                W -= np.conj(M[n - 1, m - 1]) * t
            if m + 1 <= n - 1:
                W += M[n - 1, m + 1] * np.conj(t)
    return phi0 + 2 * phi1, np.array([-W.real, -W.imag, dz0 + 2 * dz1])


def test_addition_theorem():
    rng = np.random.default_rng(1)
    for _ in range(5):
        y = rng.normal(size=3) * 0.4
        x = rng.normal(size=3) + np.array([3.0, -2.0, 2.5])
        P = 30
        U, T = regular(P, y), irregular(P, x)
        s = sum(np.conj(at(U, n, m)) * at(T, n, m) for n in range(P + 1) for m in range(-n, n + 1))
        assert abs(s - 1 / np.linalg.norm(x - y)) < 1e-13 and abs(s.imag) < 1e-14


def test_derivative_relations():
    """dT_n^m/dz = -T_{n+1}^m and (d/dx + i d/dy) T_n^m = -T_{n+1}^{m+1}
    (central differences)."""
    x = np.array([0.7, -1.1, 1.9])
    h = 1e-5
    P = 6
    T = irregular(P + 2, x)

    def d(a):
        e = np.zeros(3)
        e[a] = h
        return (irregular(P + 1, x + e) - irregular(P + 1, x - e)) / (2 * h)

    dx, dy, dz = d(0), d(1), d(2)
    for n in range(P):
        for m in range(n + 1):
            assert abs(dz[n, m] + T[n + 1, m]) < 1e-7 * abs(T[n + 1, m]) + 1e-12
            assert abs(dx[n, m] + 1j * dy[n, m] + T[n + 1, m + 1]) < 1e-7 * abs(T[n + 1, m + 1]) + 1e-12


@pytest.mark.parametrize("P,tol", [(4, 2e-3), (8, 1e-4), (12, 3e-6)])
def test_expansion_converges_to_direct_sums(P, tol):
    rng = np.random.default_rng(2)
    ys = rng.uniform(-1, 1, (50, 3))
    qs = rng.choice([-1.0, 1.0], 50)
    M = sum(q * regular(P, y) for y, q in zip(ys, qs))
    X = np.array([2.5, -3.0, 1.7])
    phi, E = expansion(P, M, X)
    d = X - ys
    r = np.linalg.norm(d, axis=1)
    phid = (qs / r).sum()
    Ed = (qs[:, None] * d / r[:, None] ** 3).sum(0)
    assert abs(phi - phid) < tol * abs(phid)
    assert np.linalg.norm(E - Ed) < tol * np.linalg.norm(Ed) * 10


def test_moment_shift():
    """M_n^m(c) = sum_k sum_l U_k^l(c1 - c) M_{n-k}^{m-l}(c1): exact."""
    rng = np.random.default_rng(3)
    ys = rng.uniform(-1, 1, (40, 3))
    qs = rng.normal(size=40)
    P = 8
    c1 = np.array([0.3, -0.2, 0.5])
    M1 = sum(q * regular(P, y - c1) for y, q in zip(ys, qs))
    M0 = sum(q * regular(P, y) for y, q in zip(ys, qs))
    U = regular(P, c1)
    for n in range(P + 1):
        for m in range(n + 1):
            s = sum(at(U, k, l) * at(M1, n - k, m - l) for k in range(n + 1) for l in range(-k, k + 1))
            assert abs(s - M0[n, m]) < 1e-12 * max(1.0, abs(M0).max())


def test_mirror_rule():
    """A source image mirrored in z (z -> -z + s_z, strength g) acts at x as
    the source itself at (x, y, -(z - s_z)), its field's z part mirrored."""
    rng = np.random.default_rng(4)
    ys = rng.uniform(-1, 1, (30, 3))
    qs = rng.normal(size=30)
    sz, g = 7.0, -0.94
    img = ys * np.array([1, 1, -1]) + np.array([0, 0, sz])
    x = np.array([0.4, -0.3, 12.0])
    d = x - img
    r = np.linalg.norm(d, axis=1)
    phi_img = g * (qs / r).sum()
    E_img = g * (qs[:, None] * d / r[:, None] ** 3).sum(0)
    xm = np.array([x[0], x[1], -(x[2] - sz)])
    dm = xm - ys
    rm = np.linalg.norm(dm, axis=1)
    phi_m = g * (qs / rm).sum()
    E_m = g * (qs[:, None] * dm / rm[:, None] ** 3).sum(0) * np.array([1, 1, -1])
    assert abs(phi_img - phi_m) < 1e-13 * abs(phi_img) + 1e-15
    assert np.abs(E_img - E_m).max() < 1e-13 * np.abs(E_img).max()


# ---- translation to a local expansion (the cell-cell step of an FMM) ----
# Not used by the kernels yet: the formulas a level-1 cell-cell step of the
# treecode would use, pinned here first.
# With M_n^m = sum_j q_j U_n^m(y_j - c_S) and D = c_T - c_S, the potential
# at c_T + w is sum_{a,b} L_a^b conj(U_a^b(w)) with
#   L_a^b = (-1)^a sum_{n,m} conj(M_n^m) T_{n+a}^{m+b}(D),
# from T_k^l(x - y) = sum_{a,b} conj(U_a^b(y)) T_{k+a}^{l+b}(x) (|y| < |x|)
# and U_a^b(-w) = (-1)^a U_a^b(w).  L_a^{-b} = (-1)^b conj(L_a^b).

def m2l(M, D, P):
    """L_a^b for 0 <= b <= a <= P from moments M (orders <= P) at D."""
    T = irregular(2 * P + 1, D)
    L = np.zeros((P + 1, P + 1), complex)
    for a in range(P + 1):
        for b in range(a + 1):
            L[a, b] = (-1) ** a * sum(np.conj(at(M, n, m)) * at(T, n + a, m + b)
                                      for n in range(P + 1) for m in range(-n, n + 1))
    return L


def l2p(L, w, P):
    """Potential and field (-grad) of the local expansion L at c_T + w, the
    field from dU_n^m/dz = U_{n-1}^m, (d/dx + i d/dy) U_n^m = -U_{n-1}^{m+1},
    (d/dx - i d/dy) U_n^m = U_{n-1}^{m-1}."""
    U = regular(P, w)
    phi = 0.0
    g = np.zeros(3, complex)
    for a in range(P + 1):
        for b in range(-a, a + 1):
            lab = at(L, a, b)
            phi += lab * np.conj(at(U, a, b))
            if a >= 1:
                dz = at(U, a - 1, b)
                dxp, dxm = -at(U, a - 1, b + 1), at(U, a - 1, b - 1)  # (dx + i dy) U, (dx - i dy) U
                dxu, dyu = 0.5 * (dxp + dxm), (dxp - dxm) / 2j
                g += lab * np.conj(np.array([dxu, dyu, dz]))
    return phi, -g


def _sources(seed, n=40):
    rng = np.random.default_rng(seed)
    return rng.uniform(-0.5, 0.5, (n, 3)), rng.choice([-1.0, 1.0], n)


def test_regular_derivative_relations():
    """dU_n^m/dz = U_{n-1}^m, (d/dx + i d/dy) U_n^m = -U_{n-1}^{m+1},
    (d/dx - i d/dy) U_n^m = U_{n-1}^{m-1} (central differences)."""
    h, P = 1e-6, 7
    v = np.array([0.3, -0.2, 0.4])
    U = regular(P, v)
    d = [(regular(P, v + h * e) - regular(P, v - h * e)) / (2 * h) for e in np.eye(3)]
    for n in range(1, P + 1):
        for m in range(n + 1):
            assert abs(d[2][n, m] - at(U, n - 1, m)) < 1e-9
            assert abs(d[0][n, m] + 1j * d[1][n, m] + at(U, n - 1, m + 1)) < 1e-9
            assert abs(d[0][n, m] - 1j * d[1][n, m] - at(U, n - 1, m - 1)) < 1e-9


def test_m2l_l2p_converge_to_direct_sums():
    """Moments about c_S translated to a local expansion about c_T (|c_T -
    c_S| = 4.2, both clusters of radius 0.87): potential and field at
    targets near c_T converge to the direct sums geometrically with the
    order; the potential is real and L_a^{-b} = (-1)^b conj(L_a^b)."""
    y, q = _sources(3)
    cT = np.array([3.1, -1.7, 2.2])
    x = np.random.default_rng(4).uniform(-0.5, 0.5, (8, 3)) + cT
    errs = []
    for P in (6, 10, 14):
        M = sum(qq * regular(P, yy) for yy, qq in zip(y, q))
        L = m2l(M, cT, P)
        T = irregular(2 * P + 1, cT)
        lm = (-1) ** 3 * sum(np.conj(at(M, n, m)) * at(T, n + 3, m - 2) for n in range(P + 1) for m in range(-n, n + 1))
        assert abs(lm - (-1) ** 2 * np.conj(L[3, 2])) < 1e-14
        e = 0.0
        for xx in x:
            phi, fld = l2p(L, xx - cT, P)
            d = xx - y
            r = np.linalg.norm(d, axis=1)
            phi_d = (q / r).sum()
            fld_d = (q[:, None] * d / r[:, None] ** 3).sum(0)
            assert abs(phi.imag) < 1e-12 and np.abs(fld.imag).max() < 1e-12
            e = max(e, abs(phi.real - phi_d) / abs(phi_d), np.abs(fld.real - fld_d).max() / np.abs(fld_d).max())
        errs.append(e)
    assert errs[0] < 1e-3 and errs[1] < errs[0] / 50 and errs[2] < errs[1] / 50, errs

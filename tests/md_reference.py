"""Reference integrators and observables for the MD tests, in numpy: the
short-range forces (WCA pairs by the minimum image, WCA walls), velocity
Verlet, the Nose-Hoover thermostat in the symmetric splitting, reversible
RESPA, and pair-distance counts by their definition.  The GPU tests drive
them with the oracle's Coulomb forces; tests/test_md_reference.py pins them
against plain loops, finite differences and the integrators' own
invariants on the CPU."""
import numpy as np

K6 = 2.0 ** (1.0 / 6.0)


def lattice_system(shape, box, seed, z_lo=0.0, z_hi=None, jitter=0.15):
    """Ions on a jittered lattice (no soft-sphere overlaps), +-1 charges,
    Maxwell velocities at kT = 1, unit masses."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    zl = z_lo, (box[2] if z_hi is None else z_hi)
    g = np.stack(np.meshgrid((np.arange(nx) + 0.5) / nx * box[0], (np.arange(ny) + 0.5) / ny * box[1],
                             zl[0] + (np.arange(nz) + 0.5) / nz * (zl[1] - zl[0]), indexing="ij"), -1).reshape(-1, 3)
    pos = g + rng.uniform(-jitter, jitter, g.shape)
    n = len(pos)
    q = np.where(rng.permutation(n) % 2 == 0, 1.0, -1.0)
    v = rng.normal(0.0, 1.0, (n, 3))
    v -= v.mean(0)
    return pos, q, v, np.ones(n)


def lj_numpy(x, box, slab, eps=1.0, sig=1.0, weps=0.0, wsig=1.0):
    """WCA pairs by the minimum image (and WCA walls in the slab): forces,
    energy and pair virial sum r . F, written out directly."""
    rc2 = (K6 * sig) ** 2
    d = x[:, None, :] - x[None, :, :]
    for k in range(3 if not slab else 2):
        d[..., k] -= box[k] * np.rint(d[..., k] / box[k])
    r2 = (d ** 2).sum(-1)
    np.fill_diagonal(r2, np.inf)
    m = r2 < rc2
    s6 = np.where(m, (sig * sig / np.where(m, r2, 1.0)) ** 3, 0.0)
    fr = np.where(m, 24 * eps * (2 * s6 * s6 - s6) / np.where(m, r2, 1.0), 0.0)
    f = (fr[..., None] * d).sum(1)
    e = 0.5 * np.where(m, 4 * eps * (s6 * s6 - s6) + eps, 0.0).sum()
    w = 0.5 * np.where(m, fr * np.where(m, r2, 0.0), 0.0).sum()
    if slab and weps > 0:
        for wall, sgn in ((0.0, 1.0), (box[2], -1.0)):
            dd = np.abs(x[:, 2] - wall)
            mm = dd < K6 * wsig
            s6w = np.where(mm, (wsig / np.where(mm, dd, 1.0)) ** 6, 0.0)
            f[:, 2] += sgn * np.where(mm, 24 * weps * (2 * s6w * s6w - s6w) / np.where(mm, dd, 1.0), 0.0)
            e += np.where(mm, 4 * weps * (s6w * s6w - s6w) + weps, 0.0).sum()
    return f, e, w


def cpu_verlet(x, v, q, m, box, coulomb, dt, nsteps, slab=False, weps=0.0):
    """The same integration on the CPU with the oracle's Coulomb forces."""
    x, v = x.copy(), v.copy()
    fc, ec = coulomb(x)
    fl, el, wl = lj_numpy(x, box, slab, weps=weps)
    f = fc + fl
    rows = []
    for _ in range(nsteps):
        v = v + 0.5 * dt * f / m[:, None]
        x = x + dt * v
        for k in range(2 if slab else 3):
            x[:, k] -= box[k] * np.floor(x[:, k] / box[k])
        fc, ec = coulomb(x)
        fl, el, wl = lj_numpy(x, box, slab, weps=weps)
        f = fc + fl
        v = v + 0.5 * dt * f / m[:, None]
        ke = 0.5 * (m[:, None] * v * v).sum()
        rows.append((ec, el, ke, wl))
    return x, v, np.array(rows)


def nh_half(xi, eta, K, nf, kT, Q, dt):
    """Half a step of the Nose-Hoover chain of length one in the symmetric
    (Trotter) splitting: quarter kick of the thermostat momentum, velocity
    scale exp(-dt/2 xi), thermostat position, quarter kick.  Returns the new
    (xi, eta) and the scale."""
    xi += 0.25 * dt * (2 * K - nf * kT) / Q
    s = np.exp(-0.5 * dt * xi)
    eta += 0.5 * dt * xi
    xi += 0.25 * dt * (2 * K * s * s - nf * kT) / Q
    return xi, eta, s


def cpu_nose_hoover(x, v, q, m, box, coulomb, dt, nsteps, kT, tau, slab=False, weps=0.0):
    """NVT on the CPU: thermostat half, velocity Verlet, thermostat half,
    with the oracle's Coulomb forces.  nf = 3n - 3 (3n - 2 in the slab),
    Q = nf kT tau^2.  Rows: E_C, E_LJ, E_kin, P after the closing half;
    also the thermostat's (xi, eta, Q xi^2 / 2 + nf kT eta) per step."""
    x, v = x.copy(), v.copy()
    n = len(x)
    nf = 3 * n - (2 if slab else 3)
    Q = nf * kT * tau * tau
    xi = eta = 0.0
    fc, ec = coulomb(x)
    fl, el, wl = lj_numpy(x, box, slab, weps=weps)
    f = fc + fl
    rows, nh = [], []
    for _ in range(nsteps):
        xi, eta, s = nh_half(xi, eta, 0.5 * (m[:, None] * v * v).sum(), nf, kT, Q, dt)
        v = s * v + 0.5 * dt * f / m[:, None]
        x = x + dt * v
        for k in range(2 if slab else 3):
            x[:, k] -= box[k] * np.floor(x[:, k] / box[k])
        fc, ec = coulomb(x)
        fl, el, wl = lj_numpy(x, box, slab, weps=weps)
        f = fc + fl
        v = v + 0.5 * dt * f / m[:, None]
        xi, eta, s = nh_half(xi, eta, 0.5 * (m[:, None] * v * v).sum(), nf, kT, Q, dt)
        v = s * v
        ke = 0.5 * (m[:, None] * v * v).sum()
        pres = (2 * ke + wl + (0.0 if slab else ec)) / (3 * box.prod())
        rows.append((ec, el, ke, pres))
        nh.append((xi, eta, 0.5 * Q * xi * xi + nf * kT * eta))
    return x, v, np.array(rows), np.array(nh)


def cpu_respa(x, v, q, m, box, coulomb, dt, k, nsteps, kT=0.0, tau=0.0, slab=False, weps=0.0, wsig=1.0):
    """Reversible RESPA on the CPU with the oracle's Coulomb forces: per
    outer step, Coulomb half kicks of dt/2 around k velocity-Verlet steps of
    dt/k under the short-range forces, optionally wrapped in the
    Nose-Hoover halves.  Rows as cpu_nose_hoover's."""
    x, v = x.copy(), v.copy()
    n = len(x)
    nf = 3 * n - (2 if slab else 3)
    Q = nf * kT * tau * tau
    xi = eta = 0.0
    fc, ec = coulomb(x)
    fl, el, wl = lj_numpy(x, box, slab, weps=weps, wsig=wsig)
    rows = []
    dti = dt / k
    axes = 2 if slab else 3
    for _ in range(nsteps):
        s = 1.0
        if kT > 0:
            xi, eta, s = nh_half(xi, eta, 0.5 * (m[:, None] * v * v).sum(), nf, kT, Q, dt)
        v = s * v + 0.5 * dt * fc / m[:, None]
        for _ in range(k):
            v = v + 0.5 * dti * fl / m[:, None]
            x = x + dti * v
            x[:, :axes] -= box[:axes] * np.floor(x[:, :axes] / box[:axes])
            fl, el, wl = lj_numpy(x, box, slab, weps=weps, wsig=wsig)
            v = v + 0.5 * dti * fl / m[:, None]
        fc, ec = coulomb(x)
        v = v + 0.5 * dt * fc / m[:, None]
        if kT > 0:
            xi, eta, s = nh_half(xi, eta, 0.5 * (m[:, None] * v * v).sum(), nf, kT, Q, dt)
            v = s * v
        ke = 0.5 * (m[:, None] * v * v).sum()
        rows.append((ec, el, ke, (2 * ke + wl + (0.0 if slab else ec)) / (3 * box.prod())))
    return x, v, np.array(rows)


def min_image_diff(a, b, box, axes=3):
    d = a - b
    for k in range(axes):
        d[:, k] -= box[k] * np.rint(d[:, k] / box[k])
    return np.abs(d).max()


def rdf_numpy(x, q, box, nbins, rmax, slab):
    """Pair-distance counts by the definition: every pair i < j with both
    charges nonzero, minimum image along the periodic axes, bin floor(r /
    dr); each FP64 operation rounded on its own in the order the library
    states (numpy evaluates one operation at a time)."""
    n = len(x)
    i, j = np.triu_indices(n, 1)
    keep = (q[i] != 0) & (q[j] != 0)
    i, j = i[keep], j[keep]
    d = []
    for k in range(3):
        dk = x[i, k] - x[j, k]
        if k < 2 or not slab:
            dk = dk - box[k] * np.rint(dk * (1.0 / box[k]))
        d.append(dk)
    r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]
    m = r2 < rmax * rmax
    b = np.minimum(nbins - 1, (np.sqrt(r2[m]) / (rmax / nbins)).astype(np.int64))
    qi, qj = q[i][m], q[j][m]
    cls = np.where((qi > 0) == (qj > 0), np.where(qi > 0, 0, 2), 1)
    h = np.zeros((3, nbins), np.int64)
    np.add.at(h, (cls, b), 1)
    return h

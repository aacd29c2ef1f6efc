"""Seeded synthetic initial conditions for the MSTAR integrator workloads.

This module is shared by the GPU path's tests and benchmark and by the CPU
oracle's tests.  It only draws random numbers and places bodies; it contains
none of the integrator's arithmetic (no forces, potentials, trees or steps).
All generators use numpy's PCG64 (``numpy.random.default_rng``) so a seed fixes
every bit of the output.

Units: G = 1.  Plummer spheres are in Henon units (total mass 1, virial radius
1, E = -1/4 in expectation), obtained analytically by choosing the Plummer
scale length 3*pi/16; positions and velocities are not re-scaled numerically.

Workloads (sizes are the ones the benchmark and parity tests use):

* ``plummer(n, seed)``                 equal-mass Plummer sphere
* ``plummer_with_central_mass``        + a point mass at rest at the origin
* ``plummer_with_binary``              + an embedded eccentric point-mass binary
* ``kepler_two_body``                  an isolated Kepler binary (paper Sec. 5.1)
* ``pythagorean``                      Burrau's three-body problem (Sec. 5.2)
* ``lidov_kozai``                      hierarchical triple (Sec. 5.3)
* ``batch_subsystems``                 thousands of small independent systems
* ``hernquist(n, seed)``               equal-mass Hernquist sphere (Sec. 5.4 clusters;
                                       the Sec. 3.5 coordinate round-trip test)
* ``timing_cluster(n, seed)``          the same without hard binaries (Sec. 5.4 timing
                                       tests; the selection evaluates pair binding
                                       energies, which is input selection only)
"""
from __future__ import annotations

import math

import numpy as np

PLUMMER_HENON_SCALE = 3.0 * math.pi / 16.0


def _rng(seed):
    return np.random.default_rng(np.random.PCG64(seed))


def _isotropic(rng, k):
    """k unit vectors uniformly distributed on the sphere."""
    cth = rng.uniform(-1.0, 1.0, k)
    phi = rng.uniform(0.0, 2.0 * math.pi, k)
    sth = np.sqrt(1.0 - cth * cth)
    return np.stack([sth * np.cos(phi), sth * np.sin(phi), cth], axis=1)


def plummer(n: int, seed: int, total_mass: float = 1.0, rmax: float = 10.0):
    """Equal-mass Plummer sphere, Aarseth-Henon-Wielen (1974) sampling.

    Radii from the inverted cumulative mass, r = a (X^(-2/3) - 1)^(-1/2),
    truncated at r <= rmax*a; speeds q * v_esc(r) with q drawn by rejection
    from q^2 (1 - q^2)^(7/2); isotropic directions.  Centre of mass and its
    velocity are then moved to zero.  Returns (m, x, v) as float64 arrays of
    shapes (n,), (n, 3), (n, 3).
    """
    rng = _rng(seed)
    a = PLUMMER_HENON_SCALE
    r = np.empty(n)
    k = 0
    while k < n:
        X = rng.uniform(0.0, 1.0, n)
        X = X[X > 0.0]
        rr = 1.0 / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
        rr = rr[rr <= rmax]
        take = min(n - k, rr.size)
        r[k:k + take] = rr[:take]
        k += take
    x = _isotropic(rng, n) * (a * r)[:, None]
    q = np.empty(n)
    k = 0
    while k < n:
        qq = rng.uniform(0.0, 1.0, 2 * n)
        yy = rng.uniform(0.0, 0.1, 2 * n)
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        qq = qq[ok]
        take = min(n - k, qq.size)
        q[k:k + take] = qq[:take]
        k += take
    vesc = math.sqrt(2.0 * total_mass / a) * (1.0 + r * r) ** (-0.25)
    v = _isotropic(rng, n) * (q * vesc)[:, None]
    m = np.full(n, total_mass / n)
    x -= (m[:, None] * x).sum(0) / m.sum()
    v -= (m[:, None] * v).sum(0) / m.sum()
    return m, x, v


def plummer_with_central_mass(n: int, seed: int, m_central: float = 0.01):
    """Plummer sphere of n stars (total mass 1) plus a point mass at rest at the
    origin.  The point mass is the last body (index n)."""
    m, x, v = plummer(n, seed)
    return (np.concatenate([m, [m_central]]),
            np.concatenate([x, np.zeros((1, 3))]),
            np.concatenate([v, np.zeros((1, 3))]))


def _rotation(rng):
    """Uniformly random rotation matrix (QR of a Gaussian matrix, sign-fixed)."""
    A = rng.standard_normal((3, 3))
    Q, R = np.linalg.qr(A)
    Q = Q * np.sign(np.diag(R))[None, :]
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    return Q


def kepler_state(m_total: float, a: float, e: float, true_anomaly: float):
    """Relative position and velocity of a Kepler orbit in its own plane
    (periapsis along +x, angular momentum along +z), G = 1."""
    p = a * (1.0 - e * e)
    f = true_anomaly
    r = p / (1.0 + e * math.cos(f))
    pos = np.array([r * math.cos(f), r * math.sin(f), 0.0])
    h = math.sqrt(m_total * p)
    vel = np.array([-m_total / h * math.sin(f), m_total / h * (e + math.cos(f)), 0.0])
    return pos, vel


def _binary_members(m1, m2, rel_x, rel_v):
    M = m1 + m2
    x = np.stack([-m2 / M * rel_x, m1 / M * rel_x])
    v = np.stack([-m2 / M * rel_v, m1 / M * rel_v])
    return np.array([m1, m2]), x, v


def kepler_two_body(m1=0.5, m2=0.5, a=1.0, e=0.9, true_anomaly=math.pi, seed=None):
    """Isolated two-body system with COM at rest at the origin.  With a seed the
    orbit gets a uniformly random orientation.  Returns (m, x, v)."""
    rel_x, rel_v = kepler_state(m1 + m2, a, e, true_anomaly)
    if seed is not None:
        Q = _rotation(_rng(seed))
        rel_x, rel_v = Q @ rel_x, Q @ rel_v
    return _binary_members(m1, m2, rel_x, rel_v)


def plummer_with_binary(n: int, seed: int, m_b: float = 0.005, a: float = 1e-3,
                        e: float = 0.9):
    """Plummer sphere of n stars plus an embedded binary of two point masses m_b,
    semi-major axis a and eccentricity e, started at apocentre with a uniformly
    random orientation; binary COM at rest at the origin.  The two point masses
    are the last two bodies."""
    m, x, v = plummer(n, seed)
    rng = _rng(seed + 7919)
    rel_x, rel_v = kepler_state(2 * m_b, a, e, math.pi)
    Q = _rotation(rng)
    mb, xb, vb = _binary_members(m_b, m_b, Q @ rel_x, Q @ rel_v)
    return (np.concatenate([m, mb]), np.concatenate([x, xb]), np.concatenate([v, vb]))


def pythagorean():
    """Burrau's problem: masses 3, 4, 5 at rest at the vertices of a 3-4-5 right
    triangle with each body opposite the side of its own length (the least
    massive body faces the shortest side), COM at the origin (Sec. 5.2; in the
    paper's units 1 length unit = 10 pc)."""
    m = np.array([3.0, 4.0, 5.0])
    x = np.array([[1.0, 3.0, 0.0], [-2.0, -1.0, 0.0], [1.0, -1.0, 0.0]])
    return m, x, np.zeros((3, 3))


def lidov_kozai(i0_deg: float = 80.0, e_in: float = 1e-3, a_in: float = 1.0,
                a_out: float = 10.0, m1: float = 1.0, m2: float = 1e-6, m3: float = 1.0):
    """Hierarchical triple of Sec. 5.3 in G = 1 units (length unit 2 pc, mass
    unit 1e9 Msun): primary m1 with a test-like secondary m2 on a nearly
    circular inner orbit inclined by i0 to a circular outer orbit of the
    perturber m3.  Returns (m, x, v) with the COM at rest at the origin."""
    xi, vi = kepler_state(m1 + m2, a_in, e_in, 0.0)
    inc = math.radians(i0_deg)
    R = np.array([[1, 0, 0], [0, math.cos(inc), -math.sin(inc)], [0, math.sin(inc), math.cos(inc)]])
    xi, vi = R @ xi, R @ vi
    mi, xs, vs = _binary_members(m1, m2, xi, vi)
    xo, vo = kepler_state(m1 + m2 + m3, a_out, 0.0, 0.5 * math.pi)
    Min = m1 + m2
    M = Min + m3
    x = np.concatenate([xs - m3 / M * xo, [Min / M * xo]])
    v = np.concatenate([vs - m3 / M * vo, [Min / M * vo]])
    return np.array([m1, m2, m3]), x, v


def batch_subsystems(n_sys: int = 4096, seed: int = 401, n_min: int = 3, n_max: int = 64,
                     m_central: float = 1.0, m_star: float = 1e-5, triple_frac: float = 0.1):
    """Many independent small systems (packed CSR-style).

    Each system: a central mass at rest at the origin plus stars of mass m_star
    with radii log-uniform in [1e-3, 1], isotropic positions, speeds
    zeta*sqrt(m_central/r) with zeta ~ U[0.5, 1.2] and isotropic directions.
    A fraction triple_frac are hierarchical triples (central mass + two stars):
    inner a log-uniform in [1e-3, 1e-1], e ~ U[0, 0.3]; outer a = a_in*U[5, 10],
    e ~ U[0, 0.3]; mutual inclination ~ U[40, 90] deg; random phases.
    Returns (offsets[n_sys+1] int64, m, x, v)."""
    rng = _rng(seed)
    sizes = rng.integers(n_min, n_max + 1, n_sys)
    is_triple = rng.uniform(0.0, 1.0, n_sys) < triple_frac
    sizes[is_triple] = 3
    offsets = np.zeros(n_sys + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    ntot = int(offsets[-1])
    m = np.empty(ntot)
    x = np.empty((ntot, 3))
    v = np.empty((ntot, 3))
    for s in range(n_sys):
        o, k = int(offsets[s]), int(sizes[s])
        m[o] = m_central
        m[o + 1:o + k] = m_star
        x[o] = 0.0
        v[o] = 0.0
        if is_triple[s]:
            a_in = 10.0 ** rng.uniform(-3.0, -1.0)
            a_out = a_in * rng.uniform(5.0, 10.0)
            inc = math.radians(rng.uniform(40.0, 90.0))
            xi, vi = kepler_state(m_central + m_star, a_in, rng.uniform(0.0, 0.3),
                                  rng.uniform(0.0, 2 * math.pi))
            xo, vo = kepler_state(m_central + 2 * m_star, a_out, rng.uniform(0.0, 0.3),
                                  rng.uniform(0.0, 2 * math.pi))
            Ri = np.array([[1, 0, 0], [0, math.cos(inc), -math.sin(inc)], [0, math.sin(inc), math.cos(inc)]])
            Q = _rotation(rng)
            xi, vi = Q @ (Ri @ xi), Q @ (Ri @ vi)
            xo, vo = Q @ xo, Q @ vo
            x[o + 1], v[o + 1] = xi, vi
            x[o + 2], v[o + 2] = xo, vo
        else:
            r = 10.0 ** rng.uniform(-3.0, 0.0, k - 1)
            x[o + 1:o + k] = _isotropic(rng, k - 1) * r[:, None]
            zeta = rng.uniform(0.5, 1.2, k - 1)
            v[o + 1:o + k] = _isotropic(rng, k - 1) * (zeta * np.sqrt(m_central / r))[:, None]
        ms = m[o:o + k]
        x[o:o + k] -= (ms[:, None] * x[o:o + k]).sum(0) / ms.sum()
        v[o:o + k] -= (ms[:, None] * v[o:o + k]).sum(0) / ms.sum()
    return offsets, m, x, v


# Named workloads with the sizes used by the benchmark and the parity tests.
def workload(name: str):
    """Return (m, x, v, params) for a named workload.  params holds the GBS
    tolerance and the integration interval for that workload."""
    if name == "plummer32":
        m, x, v = plummer(32, 101)
        return m, x, v, dict(eta=1e-12, t_end=1.0)
    if name == "plummer1000_bh":
        m, x, v = plummer_with_central_mass(1000, 201)
        return m, x, v, dict(eta=1e-13, t_end=10.0)
    if name == "plummer5000_binary":
        m, x, v = plummer_with_binary(5000, 301)
        return m, x, v, dict(eta=1e-13, t_end=1.0)
    if name == "plummer10000_binary":
        m, x, v = plummer_with_binary(10000, 302)
        return m, x, v, dict(eta=1e-13, t_end=1.0)
    if name == "plummer256_bh":
        m, x, v = plummer_with_central_mass(256, 501)
        return m, x, v, dict(eta=1e-12, t_end=None)
    raise KeyError(name)


def _hernquist_df(q):
    """Hernquist (1990) isotropic distribution function up to a constant, as a
    function of q = sqrt(binding energy * a / (G M)) in [0, 1)."""
    q2 = q * q
    return (3.0 * np.arcsin(q) + q * np.sqrt(1.0 - q2) * (1.0 - 2.0 * q2) * (8.0 * q2 * q2 - 8.0 * q2 - 3.0)) \
        / (1.0 - q2) ** 2.5


def hernquist(n: int, seed: int, r_half: float = 1.0, rmax_over_rhalf: float = 100.0):
    """Equal-mass Hernquist sphere (total mass 1, G = 1) with half-mass radius
    r_half: radii from the inverse cumulative mass r^2/(r+a)^2 with
    a = r_half / (1 + sqrt 2), truncated at rmax_over_rhalf * r_half; speeds
    drawn by rejection from v^2 f(psi - v^2/2) with the isotropic distribution
    function f (Eddington inversion of the Hernquist pair, Hernquist 1990) and
    psi = 1/(r + a); isotropic directions; centre of mass at rest at the origin.
    Returns (m, x, v)."""
    rng = _rng(seed)
    a = r_half / (1.0 + math.sqrt(2.0))
    rmax = rmax_over_rhalf * r_half
    r = np.empty(n)
    k = 0
    while k < n:
        s = np.sqrt(rng.uniform(0.0, 1.0, n))
        rr = a * s / (1.0 - s)
        rr = rr[rr <= rmax]
        take = min(n - k, len(rr))
        r[k:k + take] = rr[:take]
        k += take
    x = r[:, None] * _isotropic(rng, n)
    speed = np.empty(n)
    grid = np.linspace(0.0, 1.0, 257)[1:-1]
    for i in range(n):
        psi = 1.0 / (r[i] + a)
        vesc = math.sqrt(2.0 * psi)
        vg = grid * vesc
        qg = np.sqrt((psi - 0.5 * vg * vg) * a)
        bound = 1.2 * np.max(vg * vg * _hernquist_df(qg))
        while True:
            vv = rng.uniform(0.0, vesc)
            q = math.sqrt(max(psi - 0.5 * vv * vv, 0.0) * a)
            if rng.uniform(0.0, bound) <= vv * vv * float(_hernquist_df(np.array([q]))[0]):
                speed[i] = vv
                break
    v = speed[:, None] * _isotropic(rng, n)
    m = np.full(n, 1.0 / n)
    x = x - (m[:, None] * x).sum(0)
    v = v - (m[:, None] * v).sum(0)
    return m, x, v


# The timing clusters of the paper's N-body timing tests: M = 1e7 solar masses,
# r_half = 10 pc, integrated for 0.1 Myr.  In the units used here (G = M =
# r_half = 1) the time unit is sqrt(r_half^3 / (G M)) with
# G = 4.498502151469552e-3 pc^3 / (Msun Myr^2) (from the IAU nominal solar
# GM, the parsec and the Julian year), i.e. 0.149096 Myr.
TIMING_MYR_PER_UNIT = 0.1490960142591554
TIMING_T_END = 0.1 / TIMING_MYR_PER_UNIT


def timing_sizes():
    """The 20 cluster sizes, logarithmically spaced from 10 to 10^4."""
    return [int(round(10.0 ** (1.0 + 3.0 * k / 19.0))) for k in range(20)]


def hard_binaries(m, x, v):
    """Pairs bound more tightly than the mean kinetic energy of a body: the
    pair's two-body binding energy G m_i m_j / r - mu |v_i - v_j|^2 / 2 (with
    G = 1, mu the reduced mass) at least <m v^2 / 2> over the cluster (centre
    of mass frame).  Only pairs closer than max(m)^2 / <m v^2 / 2> can qualify,
    so a k-d tree lists the candidates.  Returns a sorted list of (i, j), i < j."""
    from scipy.spatial import cKDTree
    m = np.asarray(m, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    vc = v - (m[:, None] * v).sum(0) / m.sum()
    thresh = 0.5 * float(np.mean(m * (vc * vc).sum(1)))
    cand = cKDTree(x).query_pairs(float(m.max()) ** 2 / thresh, output_type="ndarray")
    if len(cand) == 0:
        return []
    i, j = cand[:, 0], cand[:, 1]
    dx, dv = x[j] - x[i], v[j] - v[i]
    mu = m[i] * m[j] / (m[i] + m[j])
    eb = m[i] * m[j] / np.sqrt((dx * dx).sum(1)) - 0.5 * mu * (dv * dv).sum(1)
    hit = eb >= thresh
    return sorted((int(min(a, b)), int(max(a, b))) for a, b in zip(i[hit], j[hit]))


def timing_cluster(n: int, seed: int, max_draws: int = 1000):
    """A Hernquist cluster of the timing tests (``hernquist(n, ...)``, r_half = 1)
    with no hard binary: draws with seeds 1000 * seed + k, k = 0, 1, ..., until
    ``hard_binaries`` finds none.  Returns (m, x, v, k)."""
    for k in range(max_draws):
        m, x, v = hernquist(n, 1000 * seed + k)
        if not hard_binaries(m, x, v):
            return m, x, v, k
    raise RuntimeError(f"no cluster without hard binaries in {max_draws} draws (n={n}, seed={seed})")

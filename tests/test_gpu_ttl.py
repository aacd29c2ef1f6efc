"""TTL time transformation (beta != 0, the Omega function of Sec. 2.1) on the
GPU path vs the CPU oracle, through the C ABI.

Omega couples the bodies with m <= omega_mass_max (the oracle's reading of
the example Sec. 2.1 gives: a force function of the lightest bodies); the auxiliary
variable w starts at Omega and follows dw/dt = sum_i grad_i Omega . v_i.

Tolerances are those of the Newtonian stages (see test_gpu_parity.py):
  * Omega and its gradient: 1e-13 of the per-body scale
    G mo_i sum_j mo_j / r_ij^2, |dOmega/Omega| <= 1e-13; the gradient of a
    body outside the Omega set is exactly zero.
  * leapfrog / GBS step states (including w): 1e-12 of the state scale.
  * free integrations inside the predictability horizon: 1e-10.
Every GPU result is computed twice and must be bitwise identical.
"""
import sys

import numpy as np
import pytest

import ics

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2001_03180_amd as M
    c = M.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def M():
    import paper_2001_03180_amd as M
    return M


def _system(n, seed, heavy=3, factor=10.0):
    """Plummer sphere whose first `heavy` bodies are `factor` times heavier;
    the Omega set is the remaining light bodies."""
    m, x, v = ics.plummer(n, seed)
    m = m.copy()
    m[:heavy] *= factor
    return m, x, v, 1.5 * m.min()


def _state(orc, m, x, v, op):
    """MST state with B = U - T and w = Omega of the start state."""
    parent, X, V, scal = orc.build_state(m, x, v)
    rho = orc.deconstruct(parent, X)
    _, _, U, Om, _ = orc.force(m, parent, X, rho, op)
    vt = v - (m[:, None] * v).sum(0) / m.sum()
    scal[1] = U - 0.5 * (m * (vt ** 2).sum(1)).sum()
    scal[2] = Om
    return parent, X, V, scal, rho


def _oscale(mo, rho):
    n = len(mo)
    s = np.empty(n)
    for i in range(n):
        d = rho - rho[i]
        r2 = (d * d).sum(1)
        r2[i] = np.inf
        s[i] = mo[i] * (mo / r2).sum()
    return s


@pytest.mark.parametrize("n,seed", [(32, 101), (200, 7), (1001, 201)])
@pytest.mark.parametrize("nd", [0, 2])
def test_force_omega_parity(ctx, orc, M, n, seed, nd):
    m, x, v, mmax = _system(n, seed, heavy=max(3, n // 10))
    op = orc.params(beta=1.0, omega_mass_max=mmax, n_d=nd, nthreads=0)
    parent, X, V, scal, rho = _state(orc, m, x, v, op)
    say(f"force omega n={n} nd={nd}")
    p = M.params(beta=1.0, omega_mass_max=mmax, n_d=nd)
    acc, U, Om, dOm = ctx.force(m, rho, parent, X, p, omega=True)
    acc2, U2, Om2, dOm2 = ctx.force(m, rho, parent, X, p, omega=True)
    assert np.array_equal(acc, acc2) and U == U2 and Om == Om2 and np.array_equal(dOm, dOm2)
    ao, _, Uo, Omo, dOmo = orc.force(m, parent, X, rho, op)
    mo = np.where(m <= mmax, m, 0.0)
    light = mo > 0
    assert abs(Om - Omo) <= 1e-13 * Omo
    err = np.abs(dOm - dOmo).max(1)[light] / _oscale(mo, rho)[light]
    assert err.max() <= 1e-13, err.max()
    assert np.all(dOm[~light] == 0.0)
    # the Newtonian outputs do not depend on beta
    acc0, U0 = ctx.force(m, rho, parent, X, M.params(n_d=nd))
    assert np.array_equal(acc, acc0) and U == U0


def test_force_omega_off_gives_zeros(ctx, orc, M):
    m, x, v, mmax = _system(40, 3)
    parent, X, V, scal, rho = _state(orc, m, x, v, orc.params())
    acc, U, Om, dOm = ctx.force(m, rho, parent, X, M.params(), omega=True)
    assert Om == 0.0 and np.all(dOm == 0.0)


def test_force_omega_all_light_equals_U(ctx, orc, M):
    """With every body in the Omega set, Omega is U and grad_i Omega = m_i a_i."""
    m, x, v = ics.plummer(64, 12)
    parent, X, V, scal, rho = _state(orc, m, x, v, orc.params())
    acc, U, Om, dOm = ctx.force(m, rho, parent, X, M.params(beta=1.0, omega_mass_max=1.0), omega=True)
    assert abs(Om - U) <= 1e-15 * U
    assert np.abs(dOm - m[:, None] * acc).max() <= 1e-14 * np.abs(m[:, None] * acc).max()


TRIPLETS = [(0.0, 1.0, 0.0), (1.0, 1.0, 0.0), (1.0, 0.5, 0.25)]


@pytest.mark.parametrize("abg", TRIPLETS, ids=["ttl010", "mix110", "mix1_05_025"])
@pytest.mark.parametrize("n,seed,H,nsub", [(32, 101, 0.02, 3), (200, 7, 0.005, 2)])
def test_leapfrog_ttl_parity(ctx, orc, M, abg, n, seed, H, nsub):
    a, b, g = abg
    m, x, v, mmax = _system(n, seed)
    op = orc.params(alpha=a, beta=b, gamma=g, omega_mass_max=mmax)
    parent, X, V, scal, _ = _state(orc, m, x, v, op)
    say(f"leapfrog ttl {abg} n={n}")
    p = M.params(alpha=a, beta=b, gamma=g, omega_mass_max=mmax)
    Xg, Vg, sg = ctx.leapfrog(m, parent, X, V, scal, H, nsub, p)
    Xg2, Vg2, sg2 = ctx.leapfrog(m, parent, X, V, scal, H, nsub, p)
    assert np.array_equal(Xg, Xg2) and np.array_equal(Vg, Vg2) and np.array_equal(sg, sg2)
    Xo, Vo, so, nf = orc.leapfrog(m, parent, X, V, scal, H, nsub, op)
    assert np.abs(Xg - Xo).max() <= 1e-12 * np.abs(Xo).max()
    assert np.abs(Vg - Vo).max() <= 1e-12 * np.abs(Vo).max()
    assert abs(sg[0] - so[0]) <= 1e-13 * abs(so[0])
    assert abs(sg[2] - so[2]) <= 1e-12 * abs(so[2])      # w
    assert sg[2] != scal[2]                              # w moved


@pytest.mark.parametrize("abg", TRIPLETS[:2], ids=["ttl010", "mix110"])
@pytest.mark.parametrize("n,seed,H", [(32, 101, 0.05), (200, 9, 0.01)])
def test_gbs_step_ttl_parity(ctx, orc, M, abg, n, seed, H):
    a, b, g = abg
    m, x, v, mmax = _system(n, seed)
    op = orc.params(alpha=a, beta=b, gamma=g, omega_mass_max=mmax, eta=1e-12)
    parent, X, V, scal, _ = _state(orc, m, x, v, op)
    say(f"gbs_step ttl {abg} n={n} H={H}")
    p = M.params(alpha=a, beta=b, gamma=g, omega_mass_max=mmax, eta=1e-12)
    Xg, Vg, sg, acc, eps, hn = ctx.gbs_step(m, parent, X, V, scal, H, p)
    out2 = ctx.gbs_step(m, parent, X, V, scal, H, p)
    assert np.array_equal(Xg, out2[0]) and np.array_equal(sg, out2[2]) and eps == out2[4]
    Xo, Vo, so, acco, epso, hno, nf = orc.gbs_step(m, parent, X, V, scal, H, op)
    # same bound as the Newtonian GBS step: Neville weights of size ~2e2 on
    # division states that agree to ~1e-15
    eps_tol = 1e-3 * epso + 5e-13
    assert abs(eps - epso) <= eps_tol, (eps, epso)
    if abs(epso - 1e-12) > eps_tol:
        assert acc == acco
    if acc and acco:
        assert np.abs(Xg - Xo).max() <= 1e-12 * np.abs(Xo).max()
        assert np.abs(Vg - Vo).max() <= 1e-12 * np.abs(Vo).max()
        assert abs(sg[0] - so[0]) <= 1e-14 * abs(so[0]) + 1e-16
        assert abs(sg[2] - so[2]) <= 1e-12 * abs(so[2])
    elif not acc:
        assert np.array_equal(Xg, X) and hn == 0.5 * H


def _rel_state_err(xg, vg, xo, vo, m):
    rc = (m[:, None] * xo).sum(0) / m.sum()
    vc = (m[:, None] * vo).sum(0) / m.sum()
    return np.abs(xg - xo).max() / np.abs(xo - rc).max(), np.abs(vg - vo).max() / np.abs(vo - vc).max()


@pytest.mark.parametrize("abg,t_end", [((0.0, 1.0, 0.0), 0.1), ((1.0, 1.0, 0.0), 0.1)], ids=["ttl010", "mix110"])
def test_integrate_ttl_parity(ctx, orc, M, abg, t_end):
    a, b, g = abg
    m, x, v, mmax = _system(10, 41)
    say(f"integrate ttl {abg} t_end={t_end}")
    p = M.params(alpha=a, beta=b, gamma=g, omega_mass_max=mmax, eta=1e-11)
    xg, vg, rc, st = ctx.integrate(m, x, v, 0.0, t_end, p)
    xg2, vg2, _, _ = ctx.integrate(m, x, v, 0.0, t_end, p)
    assert np.array_equal(xg, xg2) and np.array_equal(vg, vg2)
    xo, vo, rco, sto = orc.integrate(m, x, v, 0.0, t_end,
                                     orc.params(alpha=a, beta=b, gamma=g, omega_mass_max=mmax, eta=1e-11))
    assert rc == rco == 0
    assert abs(st["t_reached"] - sto["t_reached"]) <= 2e-14 * t_end
    ex, ev = _rel_state_err(xg, vg, xo, vo, m)
    assert ex <= 1e-10 and ev <= 1e-10, (ex, ev)
    d0, dg = orc.diagnostics(m, x, v), orc.diagnostics(m, xg, vg)
    assert abs((dg["E"] - d0["E"]) / d0["E"]) < 1e-10


def test_ttl_needs_omega_bodies(ctx, M):
    m, x, v, _ = _system(10, 41)
    with pytest.raises(M.MstarError) as e:
        ctx.integrate(m, x, v, 0.0, 0.1, M.params(alpha=0.0, beta=1.0, gamma=0.0, omega_mass_max=0.0))
    assert e.value.code == M.E_INVAL
    with pytest.raises(M.MstarError) as e:
        ctx.integrate(m, x, v, 0.0, 0.1, M.params(beta=-1.0))
    assert e.value.code == M.E_INVAL

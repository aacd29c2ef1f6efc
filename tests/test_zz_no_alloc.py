"""mstar_force_noalloc (the allocation-free force evaluation) against the
existing entry point mstar_force, through the C ABI, from the largest size
the scratch array takes down to 65 bodies.

Same bar as the force parity tests: max_i |a_i - a_i'| / (G sum_j m_j/r_ij^2)
<= 1e-13 and |U - U'| <= 1e-13 U, here also against the oracle.  Two calls in
a row, the second with a smaller N (the scratch array keeps the first call's
contents), each checked; a call beyond the size limit is refused; a parent
array that is not a tree gives NaN outputs; the call records into a HIP graph
and replays with eager work between replays.
"""
import sys

import numpy as np
import pytest

import ics

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)
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


def _case(orc, n, seed):
    if n > 1000:
        m, x, v = ics.plummer_with_binary(n - 2, seed)
    else:
        m, x, v = ics.plummer(n, seed)
    parent, X, V, scal = orc.build_state(m, x, v)
    rho = orc.deconstruct(parent, X)
    return m, rho, parent, X


def _scale(m, rho):
    s = np.empty(len(m))
    for i in range(len(m)):
        d = rho - rho[i]
        r2 = (d * d).sum(1)
        r2[i] = np.inf
        s[i] = (m / r2).sum()
    return s


def _noalloc(M, m, rho, parent, X, nd):
    import torch
    T = lambda a, dt=torch.float64: torch.tensor(a, dtype=dt, device="cuda")
    acc = torch.full((len(m), 3), -1.0, dtype=torch.float64, device="cuda")
    U = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    rc = M.force_noalloc(T(m), T(rho), T(parent, torch.int32), T(X), acc, U, M.params(n_d=nd))
    torch.cuda.synchronize()
    return rc, acc.cpu().numpy(), float(U.cpu()[0])


@pytest.mark.parametrize("nd", [2, 0])
def test_noalloc_matches_force_twice_shrinking(ctx, orc, nd):
    import paper_2001_03180_amd as M
    # the largest size the scratch array takes first, then smaller ones
    for n, seed in ((M.NOALLOC_MAX_N, 17), (5002, 301), (1001, 201), (65, 3)):
        m, rho, parent, X = _case(orc, n, seed)
        say(f"force_noalloc n={n} nd={nd}")
        rc, acc, U = _noalloc(M, m, rho, parent, X, nd)
        assert rc == M.OK
        a_ref, U_ref = ctx.force(m, rho, parent, X, M.params(n_d=nd))
        sc = _scale(m, rho)
        assert (np.abs(acc - a_ref).max(1) / sc).max() <= 1e-13
        assert abs(U - U_ref) <= 1e-13 * U_ref
        ao, _, Uo, _, _ = orc.force(m, parent, X, rho, orc.params(n_d=nd, nthreads=0))
        assert (np.abs(acc - ao).max(1) / sc).max() <= 1e-13
        assert abs(U - Uo) <= 1e-13 * Uo
        rc2, acc2, U2 = _noalloc(M, m, rho, parent, X, nd)
        assert rc2 == M.OK and np.array_equal(acc, acc2) and U == U2


def test_noalloc_limits_and_bad_trees(ctx, orc):
    import torch
    import paper_2001_03180_amd as M
    n = M.NOALLOC_MAX_N + 1
    z = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    rc = M.force_noalloc(torch.ones(n, dtype=torch.float64, device="cuda"), z, torch.zeros(n, dtype=torch.int32,
                         device="cuda"), z, z.clone(), torch.zeros(1, dtype=torch.float64, device="cuda"))
    assert rc == M.E_INVAL
    m, rho, parent, X = _case(orc, 200, 7)
    rc = M.force_noalloc(*(torch.tensor(a, device="cuda") for a in (m, rho)),
                         torch.tensor(parent, dtype=torch.int32, device="cuda"), torch.tensor(X, device="cuda"),
                         torch.zeros((200, 3), dtype=torch.float64, device="cuda"),
                         torch.zeros(1, dtype=torch.float64, device="cuda"), M.params(beta=1.0))
    assert rc == M.E_UNSUPPORTED
    for what, bad in (("index out of range", lambda p: np.where(p == p.max(), 10 ** 6, p)),
                      ("two roots", lambda p: np.where(np.arange(len(p)) == 5, -1, p)),
                      ("cycle", lambda p: _cycle(p))):
        say(f"bad tree: {what}")
        rc, acc, U = _noalloc(M, m, rho, bad(parent.copy()).astype(np.int32), X, 2)
        assert rc == M.OK and np.isnan(acc).all() and np.isnan(U)
    rc, acc, U = _noalloc(M, m, rho, parent, X, 2)   # and a good one after them
    a_ref, U_ref = ctx.force(m, rho, parent, X, M.params(n_d=2))
    assert (np.abs(acc - a_ref).max(1) / _scale(m, rho)).max() <= 1e-13 and abs(U - U_ref) <= 1e-13 * U_ref


def _cycle(p):
    """Point the root at a grandchild of itself: no root, a cycle."""
    r = int(np.nonzero(p < 0)[0][0])
    kids = np.nonzero(p == r)[0]
    for k in kids:
        gk = np.nonzero(p == k)[0]
        if len(gk):
            p[r] = gk[0]
            return p
    p[r] = kids[0]
    return p


def test_noalloc_in_a_graph(ctx, orc):
    """Captured into a HIP graph (no allocation happens inside the capture) and
    replayed three times, with the inputs changed and eager work between the
    replays; every replay equals an eager call on the same inputs."""
    import torch
    import paper_2001_03180_amd as M
    m, rho, parent, X = _case(orc, 1001, 201)
    dm, dr, dp, dX = (torch.tensor(m, device="cuda"), torch.tensor(rho, device="cuda"),
                      torch.tensor(parent, dtype=torch.int32, device="cuda"), torch.tensor(X, device="cuda"))
    acc = torch.zeros((1001, 3), dtype=torch.float64, device="cuda")
    U = torch.zeros(1, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        assert M.force_noalloc(dm, dr, dp, dX, acc, U, M.params(), stream=s) == M.OK   # first call: set-up
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        assert M.force_noalloc(dm, dr, dp, dX, acc, U, M.params(), stream=s) == M.OK
    for r in range(3):
        say(f"graph replay {r}")
        scale = 1.0 + 0.01 * r
        dr.copy_(torch.tensor(rho * scale, device="cuda"))
        dX.copy_(torch.tensor(X * scale, device="cuda"))
        g.replay()
        torch.cuda.synchronize()
        got_a, got_U = acc.cpu().numpy().copy(), float(U.cpu()[0])
        junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64).sum()
        torch.cuda.synchronize()
        assert np.isfinite(float(junk))
        rc, want_a, want_U = _noalloc(M, m, rho * scale, parent, X * scale, 2)
        assert np.array_equal(got_a, want_a) and got_U == want_U

"""The driver replays each GBS step attempt from a captured HIP graph; with
MSTAR_EAGER it launches the same kernels from the host.  The two must give
bitwise identical integrations: every attempt is a replay, with the driver's
own eager work (MST rebuilds, control read-backs) between replays, and a
change of parameters, end time, N or field must recapture."""
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


def _same(a, b):
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2] == b[2]
    assert a[3] == b[3]


def test_graph_replay_matches_eager(ctx, M):
    m, x, v, _ = ics.workload("plummer32")
    say("graph vs eager, plummer32 t=0.3")
    g = ctx.integrate(m, x, v, 0.0, 0.3, M.params(eta=1e-12))
    e = ctx.integrate(m, x, v, 0.0, 0.3, M.params(eta=1e-12, flags=M.EAGER))
    assert g[3]["steps_accepted"] + g[3]["steps_rejected"] > 10
    _same(g, e)


def test_graph_recaptures_on_changes(ctx, M):
    """Alternating sizes, end times, tolerances and the external field on one
    context: each graph result equals its eager counterpart."""
    cases = [(ics.workload("plummer32")[:3], 0.1, dict(eta=1e-12), None),
             (ics.plummer(64, 5), 0.05, dict(eta=1e-12), None),
             (ics.workload("plummer32")[:3], 0.2, dict(eta=1e-11), None),
             (ics.workload("plummer32")[:3], 0.2, dict(eta=1e-11), [[5.0, 4.0, 0.0, 0.0, 0.5]]),
             (ics.plummer(64, 5), 0.05, dict(eta=1e-12, n_d=3), None),
             (ics.workload("plummer32")[:3], 0.1, dict(eta=1e-12), None)]
    for (m, x, v), T, kw, pts in cases:
        say(f"recapture N={len(m)} T={T} {kw} field={pts is not None}")
        if pts is None:
            g = ctx.integrate(m, x, v, 0.0, T, M.params(**kw))
            e = ctx.integrate(m, x, v, 0.0, T, M.params(flags=M.EAGER, **kw))
        else:
            g = ctx.integrate_ext(m, x, v, 0.0, T, points=pts, p=M.params(**kw))
            e = ctx.integrate_ext(m, x, v, 0.0, T, points=pts, p=M.params(flags=M.EAGER, **kw))
        _same(g, e)


def test_graph_ttl_and_device_pointers(ctx, M):
    import torch
    m, x, v = ics.plummer(48, 9)
    kw = dict(eta=1e-12, alpha=1.0, beta=1.0, gamma=0.0, omega_mass_max=1.0)
    say("graph vs eager, TTL, device pointers")
    e = ctx.integrate(m, x, v, 0.0, 0.05, M.params(flags=M.EAGER, **kw))
    g = ctx.integrate(torch.tensor(m, device="cuda"), torch.tensor(x, device="cuda"),
                      torch.tensor(v, device="cuda"), 0.0, 0.05, M.params(**kw))
    assert np.array_equal(g[0].cpu().numpy(), e[0]) and np.array_equal(g[1].cpu().numpy(), e[1])
    assert g[3] == e[3]


def test_unfinished_rebuild_repeats_the_step_exactly(M):
    """A rebuild queued with no spare Borůvka round often does not finish; the
    step taken on the old tree is then discarded, the tree completed and the
    step repeated.  The integration must equal the default one bit for bit
    (only the count of force evaluations grows)."""
    import os
    import torch
    if not torch.cuda.is_available():   # torch first: it brings up the device runtime
        pytest.skip("no GPU")
    m, x, v = ics.plummer_with_central_mass(256, 501)
    p = dict(eta=1e-12)
    ref = M.Context(0)
    try:
        say("spare rounds 1 (default), N=257, t=0.5")
        a = ref.integrate(m, x, v, 0.0, 0.5, M.params(**p))
    finally:
        ref.close()
    os.environ["MSTAR_MST_SPARE_ROUNDS"] = "0"
    try:
        c = M.Context(0)
    finally:
        del os.environ["MSTAR_MST_SPARE_ROUNDS"]
    try:
        say("spare rounds 0, N=257, t=0.5")
        b = c.integrate(m, x, v, 0.0, 0.5, M.params(**p))
        e = c.integrate(m, x, v, 0.0, 0.5, M.params(flags=M.EAGER, **p))
    finally:
        c.close()
    assert a[3]["steps_accepted"] > 20
    # the repeat path ran: each repeat re-evaluates a whole attempt
    assert b[3]["force_evals"] > a[3]["force_evals"] and e[3]["force_evals"] == b[3]["force_evals"]
    for r in (b, e):
        assert np.array_equal(a[0], r[0]) and np.array_equal(a[1], r[1])
        for k in ("steps_accepted", "steps_rejected", "mst_rebuilds", "t_reached"):
            assert a[3][k] == r[3][k], k


def test_two_division_chains(M):
    """With MSTAR_DIV_CHAINS=0 the divisions at N_p = 5002 run as two chains
    of launches on two streams (automatic where the mutual kernel runs at
    N >= 4096).  Graph replay, which captures the fork and the join, equals
    eager launch bit for bit.  Against one chain (the default) the force
    launches group the
    evaluations and their partials differently, so the agreement is to
    rounding: the step lengths differ in their last bits, and the end-time
    iteration may take a step more or less; both reach t_end, with end states
    within 1e-10 of the system's extent and the same energy error to 1e-13."""
    import os
    import torch
    if not torch.cuda.is_available():   # torch first: it brings up the device runtime
        pytest.skip("no GPU")
    from bench import _energy
    m, x, v, _ = ics.workload("plummer5000_binary")
    te = 2e-3
    p = dict(eta=1e-13)
    one = M.Context(0)
    old = os.environ.get("MSTAR_DIV_CHAINS")
    os.environ["MSTAR_DIV_CHAINS"] = "0"
    try:
        two = M.Context(0)
    finally:
        if old is None:
            os.environ.pop("MSTAR_DIV_CHAINS", None)
        else:
            os.environ["MSTAR_DIV_CHAINS"] = old
    try:
        say("plummer5000_binary to t=2e-3: one chain, two chains (graph), two chains (eager)")
        a = one.integrate(m, x, v, 0.0, te, M.params(**p))
        g = two.integrate(m, x, v, 0.0, te, M.params(**p))
        e = two.integrate(m, x, v, 0.0, te, M.params(flags=M.EAGER, **p))
        assert g[3]["steps_accepted"] + g[3]["steps_rejected"] > 10
        _same(g, e)
        say(f"steps (accepted + rejected): one chain {a[3]['steps_accepted']} + {a[3]['steps_rejected']}, "
            f"two chains {g[3]['steps_accepted']} + {g[3]['steps_rejected']}")
        assert abs(g[3]["steps_accepted"] - a[3]["steps_accepted"]) <= 2
        for r in (a, g):
            assert abs(r[3]["t_reached"] - te) <= 1e-12 * te
        ext = np.ptp(a[0], axis=0).max()
        dx = np.abs(g[0] - a[0]).max() / ext
        dv = np.abs(g[1] - a[1]).max() / np.ptp(a[1], axis=0).max()
        e0 = _energy(m, x, v)
        de = abs(_energy(m, g[0], g[1]) / e0 - _energy(m, a[0], a[1]) / e0)
        say(f"state difference {dx:.2e} (x), {dv:.2e} (v) of the extents; dE/E difference {de:.1e}")
        assert dx <= 1e-10 and dv <= 1e-10 and de <= 1e-13
    finally:
        one.close()
        two.close()


@pytest.mark.parametrize("case", ["ttl", "field"])
def test_two_chains_with_ttl_and_external_field(M, case):
    """MSTAR_DIV_CHAINS=2 with the pairwise kernel: the TTL run (Omega partials
    per slot) and a run under an external field (per-slot field kicks).  Graph
    replay equals eager launch bit for bit; against one chain the agreement is
    to rounding (end states within 1e-10 of the extents)."""
    import os
    import torch
    if not torch.cuda.is_available():   # torch first: it brings up the device runtime
        pytest.skip("no GPU")
    m, x, v = ics.plummer(48, 9)
    one = M.Context(0)
    old = os.environ.get("MSTAR_DIV_CHAINS")
    os.environ["MSTAR_DIV_CHAINS"] = "2"
    try:
        two = M.Context(0)
    finally:
        if old is None:
            os.environ.pop("MSTAR_DIV_CHAINS", None)
        else:
            os.environ["MSTAR_DIV_CHAINS"] = old
    if case == "ttl":
        kw = dict(eta=1e-12, alpha=1.0, beta=1.0, gamma=0.0, omega_mass_max=1.0)

        def run(c, **f):
            return c.integrate(m, x, v, 0.0, 0.05, M.params(**kw, **f))
    else:
        kw = dict(eta=1e-12)

        def run(c, **f):
            return c.integrate_ext(m, x, v, 0.0, 0.05, g=(0.3, 0.0, 0.1), points=[[5.0, 4.0, 0.0, 0.0, 0.5]],
                                   p=M.params(**kw, **f))
    try:
        say(f"two chains, {case}: one chain, two chains (graph), two chains (eager)")
        a = run(one)
        b = run(two)
        e = run(two, flags=M.EAGER)
        assert b[3]["steps_accepted"] + b[3]["steps_rejected"] > 5
        _same(b, e)
        assert abs(b[3]["steps_accepted"] - a[3]["steps_accepted"]) <= 2
        dx = np.abs(b[0] - a[0]).max() / np.ptp(a[0], axis=0).max()
        dv = np.abs(b[1] - a[1]).max() / np.ptp(a[1], axis=0).max()
        say(f"state difference {dx:.2e} (x), {dv:.2e} (v) of the extents")
        assert dx <= 1e-10 and dv <= 1e-10
    finally:
        one.close()
        two.close()

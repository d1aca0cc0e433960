"""Batched ensemble of 1D problems (grmhd_batch_*) against the oracle run on
each problem alone.

FP64 bar: relative L1 <= 1e-10 per problem (the oracle and the batch kernel
evaluate the same scheme in different operation orders).  Mixed: <= 1e-5 on
the physical variables.  The launch shape and the LDS/global choice change
which thread computes a face, not what it computes, so results are
bitwise independent of them."""
import sys

import numpy as np
import pytest
import torch

from paper_1102_5202_amd import workloads as WL

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def G():
    from paper_1102_5202_amd import grmhd
    grmhd.load()
    return grmhd


def _oracle_problem(orc, e, b):
    w = e.problem(b)
    pb = orc.Problem(**w.problem_kwargs())
    U0 = orc.prim2con(pb, w.P)
    U, P, st = orc.step(pb, U0, w.P, w.dt, w.nsteps)
    return U.reshape(9, -1), P.reshape(9, -1)


@pytest.mark.parametrize("bc,split", [(WL.OUTFLOW, False), (WL.PERIODIC, False), (WL.OUTFLOW, True),
                                      (WL.PERIODIC, True)])
def test_batch_matches_oracle(G, orc, bc, split):
    """Every problem against the oracle run alone; with split, the work
    spread over co-resident workgroups (the longer problems divided into
    parts whose end cells cross between workgroups, periodic ends joining a
    problem's first and last part)."""
    e = WL.config5(nprob=12, nmin=20, nmax=150, k=1)
    e.bc = bc
    s = G.batch_for(e, device=DEV)
    if split:
        s.set_shape(256, 2)
    P0 = s.pack(e.P)
    U = s.cons(P0)
    s.evolve(U)
    P = s.prim(U)
    st = s.status()
    Us, Ps = s.unpack(U.cpu()), s.unpack(P.cpu())
    worst = 0.0
    for b in range(e.n.__len__()):
        Ur, Pr = _oracle_problem(orc, e, b)
        err = orc.parity_error(Us[b].numpy(), Ur)
        worst = max(worst, float(err[:8].max()))
        assert np.all(err[:8] <= 1e-10), (b, e.n[b], err)
        assert np.all(Us[b][8].numpy() == 0.0)
    say("batch bc=%d worst rel-L1 %.3g" % (bc, worst), st)


def test_batch_chunked_equals_one_shot_and_shapes_agree(G):
    """Evolving in chunks of steps equals one call, bitwise.  Every launch
    shape computes the same scheme; the separately compiled kernel instances
    may contract different multiply-adds into FMAs, so shapes agree to
    rounding (relative L1 <= 1e-13), not bitwise.  The tuner's trial runs
    leave the state alone."""
    e = WL.config5(nprob=9, nmin=30, nmax=300, k=2)
    ref = None
    for chunk in (None, 7):
        s = G.batch_for(e, device=DEV)
        U = s.cons(s.pack(e.P))
        if chunk is None:
            s.evolve(U)
        else:
            for _ in range(max(e.steps) // chunk + 1):
                s.evolve(U, chunk)
        out = U.cpu().numpy()
        if ref is None:
            ref = out
        assert np.array_equal(out, ref)
    for th, lds in [(t, l) for t in (256, 512, 1024) for l in (0, 1)] + [(256, 2)]:
        if True:
            s = G.batch_for(e, device=DEV)
            s.set_shape(th, lds)
            U = s.cons(s.pack(e.P))
            s.evolve(U)
            rel = np.abs(U.cpu().numpy() - ref).sum() / np.abs(ref).sum()
            say("shape", th, lds, "rel-L1 vs default", rel)
            assert rel <= 1e-13
    s = G.batch_for(e, device=DEV)
    U = s.cons(s.pack(e.P))
    U0 = U.clone()
    th, lds = s.tune(U, trial_steps=5)
    assert torch.equal(U, U0)
    say("tuned shape", th, lds)


@pytest.mark.parametrize("precision,lds", [("fp64", 0), ("fp64", 1), ("mixed", 1), ("fp64", 2), ("mixed", 2)])
def test_batch_graph_replay_matches_eager(G, precision, lds):
    """One persistent launch of a chunk of steps (for split problems, the
    flag set-up and the launch) captured in a HIP graph and replayed several
    times (eager work and synchronisation between the replays) equals the same
    chunks run eagerly, bitwise, with the rows in HBM, in LDS and split."""
    e = WL.config5(nprob=7, nmin=40, nmax=260, k=3)
    th = 256 if lds == 2 else 512
    se = G.batch_for(e, device=DEV, precision=precision)
    se.set_shape(th, lds)
    Ue = se.cons(se.pack(e.P))
    sg = G.batch_for(e, device=DEV, precision=precision)
    sg.set_shape(th, lds)
    Ug = sg.cons(sg.pack(e.P))
    torch.cuda.synchronize()
    chunk = 11
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sg.set_stream(torch.cuda.current_stream())
        sg.evolve(Ug, chunk)
    sg.set_stream(torch.cuda.current_stream())
    for r in range(4):
        g.replay()
        torch.cuda.synchronize()
        se.evolve(Ue, chunk)
        torch.cuda.synchronize()
        assert torch.equal(Ug, Ue), r
    say(precision, "graph replays match eager; status", sg.status())


_full = {}


def _full_size_states(G):
    """Config 5 at full size evolved in FP64 and mixed (tuned launch shapes),
    once per module."""
    if not _full:
        e = WL.config5()
        for prec in ("fp64", "mixed"):
            s = G.batch_for(e, device=DEV, precision=prec)
            U = s.cons(s.pack(e.P))
            th, lds = s.tune(U, trial_steps=20)
            s.evolve(U)
            torch.cuda.synchronize()
            say(prec, "tuned", th, lds, s.status())
            assert bool(torch.isfinite(U).all())
            _full[prec] = [x.numpy() for x in s.unpack(U.cpu())]
        _full["e"] = e
    return _full


def test_batch_full_size_sampled(G, orc):
    """The ensemble at full size (256 problems, 200..4000 cells, each to
    t = 0.4): every state finite, the three smallest problems against the
    oracle at the FP64 bar."""
    res = _full_size_states(G)
    e = res["e"]
    for b in np.argsort(e.n)[:3]:
        Ur, _ = _oracle_problem(orc, e, int(b))
        err = orc.parity_error(res["fp64"][b], Ur)
        say("problem", b, "n", e.n[b], "rel-L1", err.max())
        assert np.all(err <= 1e-10)


@pytest.mark.xfail(strict=True, reason="discontinuous 1D solutions: FP32 face arithmetic moves sub-cell "
                                       "features, so the longer problems end 1e-5 .. 1e-3 from FP64")
def test_batch_full_size_mixed_within_1e5(G, orc):
    """Mixed against FP64 (itself matched to the oracle) on every problem of
    the full ensemble, all nine variables, at the 1e-5 bar.  It fails on the
    longer problems; the distribution is reported."""
    res = _full_size_states(G)
    e = res["e"]
    errs = np.array([orc.parity_error(res["mixed"][b], res["fp64"][b]) for b in range(len(e.n))])
    worst = errs.max(axis=1)
    order = np.argsort(worst)[::-1]
    say("mixed vs fp64 per-problem rel-L1 (all variables): median %.2e, 90%% %.2e, worst %.2e, above 1e-5: %d"
        % (np.median(worst), np.percentile(worst, 90), worst.max(), int((worst > 1e-5).sum())))
    for b in order[:6]:
        say("  problem", b, "n", e.n[b], "by variable", np.array2string(errs[b], precision=2))
    assert np.all(worst <= 1e-5)


def test_batch_one_unknown_recovery(G, orc):
    """The ensemble with the recovery's one-unknown iteration: the same root,
    the same bar against the oracle."""
    e = WL.config5(nprob=6, nmin=20, nmax=150, k=3)
    s = G.batch_for(e, device=DEV, recovery="1d")
    U = s.cons(s.pack(e.P))
    s.evolve(U)
    Us = s.unpack(U.cpu())
    for b in range(len(e.n)):
        Ur, _ = _oracle_problem(orc, e, b)
        err = orc.parity_error(Us[b].numpy(), Ur)
        assert np.all(err[:8] <= 1e-10), (b, err)


def test_batch_busy_fraction(G):
    """The busy fraction of the last launch, from the workgroups' clock
    readings: in (0, 1], and near 1 for an ensemble of equal problems on one
    workgroup per problem (every slot works until the end)."""
    e = WL.config5(nprob=12, nmin=100, nmax=101, k=4)
    for lds in (0, 2):
        s = G.batch_for(e, device=DEV)
        s.set_shape(256, lds)
        U = s.cons(s.pack(e.P))
        s.evolve(U)
        busy, slots = s.busy()
        say("placement", lds, "busy", busy, "slots", slots)
        assert 0.0 < busy <= 1.0 + 1e-12
        assert 1 <= slots
        if lds == 0:
            assert slots == len(e.n) and busy > 0.5


def test_batch_split_packs_small_problems(G, orc):
    """Two large problems and many small ones: with the rows split among
    workgroups the large problems are divided into parts and the small ones
    packed whole into shared workgroups (run one after another).  The result
    matches one workgroup per problem to rounding (relative L1 <= 1e-12: the
    separately compiled kernels contract multiply-adds differently, and the
    two large problems take 1500 steps of a discontinuous solution), and the
    oracle on a large and a few small problems."""
    small = WL.config5(nprob=120, nmin=20, nmax=40, k=5)
    big = WL.config5(nprob=2, nmin=1500, nmax=1600, k=6)
    # the two large problems in front of the small ones
    e = WL.Ensemble(name="packed", P=list(big.P) + list(small.P), n=list(big.n) + list(small.n),
                    dt=list(big.dt) + list(small.dt), steps=list(big.steps) + list(small.steps))
    res = {}
    for lds in (2, 0):
        s = G.batch_for(e, device=DEV)
        s.set_shape(256, lds)
        U = s.cons(s.pack(e.P))
        s.evolve(U)
        busy, slots = s.busy()
        st = s.status()
        say("placement", lds, "workgroups", slots, "busy", busy, st)
        res[lds] = U.cpu().numpy()
    rel = np.abs(res[2] - res[0]).sum() / np.abs(res[0]).sum()
    say("split+packed vs one workgroup per problem: rel-L1", rel)
    assert rel <= 1e-12
    s = G.batch_for(e, device=DEV)
    Us = s.unpack(torch.from_numpy(res[2]))
    for b in (0, 2, 3, len(e.n) - 1):
        Ur, _ = _oracle_problem(orc, e, b)
        err = orc.parity_error(Us[b].numpy(), Ur)
        assert np.all(err[:8] <= 1e-10), (b, err)


def test_batch_split_multichunk_matches_oracle(G, orc):
    """The full ensemble with the split placement: a problem packed whole of
    about 1,000 cells and one split into parts of several hundred cells both
    walk their cells in several chunks of 255 per substep; each matches the
    oracle run alone at the FP64 bar."""
    e = WL.config5()
    s = G.batch_for(e, device=DEV)
    s.set_shape(256, 2)
    U = s.cons(s.pack(e.P))
    s.evolve(U)
    st = s.status()
    Us = s.unpack(U.cpu())
    n = np.array(e.n)
    for target in (1000, 1500):
        b = int(np.argmin(np.abs(n - target)))
        Ur, _ = _oracle_problem(orc, e, b)
        err = orc.parity_error(Us[b].numpy(), Ur)
        say("split, problem", b, "n", e.n[b], "rel-L1", err.max(), st)
        assert np.all(err <= 1e-10), (b, err)

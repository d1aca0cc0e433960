"""grmhd_rhs_noalloc, the entry point that allocates nothing (its scratch is
the library's static device array), against grmhd_rhs through a context with
a torch-owned workspace: bitwise the same right-hand side on two calls in a
row, the second on a smaller grid (the scratch keeps the first call's
contents), in both precisions; a grid whose workspace exceeds the scratch is
refused."""
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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_rhs_noalloc_matches_rhs_on_two_calls(precision):
    from paper_1102_5202_amd import grmhd
    grmhd.load()
    cases = (WL.config3(n=(40, 36, 34), nsteps=0), WL.config2(n=(21, 18, 13), nsteps=0))
    for w in cases:
        say("rhs_noalloc %s %s" % (precision, w.n))
        P = torch.from_numpy(np.ascontiguousarray(w.P)).to(DEV)
        R_ref = grmhd.solver_for(w, device=DEV, precision=precision).rhs(P)
        R = grmhd.rhs_noalloc_for(w, P, precision=precision)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(R).all())
        assert torch.equal(R, R_ref)


def test_rhs_noalloc_refuses_a_grid_past_its_scratch():
    from paper_1102_5202_amd import grmhd
    w = WL.config2(n=64, nsteps=0)
    assert grmhd.workspace_bytes(w.n, w.lo, w.hi, w.bc) > grmhd.NOALLOC_SCRATCH_BYTES
    P = torch.from_numpy(np.ascontiguousarray(w.P)).to(DEV)
    with pytest.raises(RuntimeError, match="workspace"):
        grmhd.rhs_noalloc_for(w, P)

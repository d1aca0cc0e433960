"""The library's compiled device arithmetic (grmhd_device_arith: FP64 division,
square root and reciprocal square root as the kernels evaluate them, with the
device build's reciprocal and approximate-function flags) against correctly
rounded results on seeded operands spread over 80 binades: division within 2
ulp, square root within 1 ulp, reciprocal square root within 2 ulp; exact
cases stay exact."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def ulps(got, ref):
    return np.abs(got - ref) / np.spacing(np.abs(ref))


def test_division_sqrt_rsqrt_against_correct_rounding():
    from paper_1102_5202_amd import grmhd
    grmhd.load()
    rng = np.random.default_rng(11025202 + 77)
    n = 1 << 20
    x = 10.0 ** rng.uniform(-12.0, 12.0, n) * rng.uniform(1.0, 2.0, n)
    y = 10.0 ** rng.uniform(-12.0, 12.0, n) * rng.choice([-1.0, 1.0], n)
    out = grmhd.device_arith(torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV)).cpu().numpy()
    div, sq, rsq = out
    ref_div = x / y                                   # IEEE double division: correctly rounded
    ref_sq = np.sqrt(x)                               # correctly rounded
    ref_rsq = (1.0 / np.sqrt(x.astype(np.longdouble))).astype(np.float64)
    e_div, e_sq, e_rsq = ulps(div, ref_div), ulps(sq, ref_sq), ulps(rsq, ref_rsq)
    print("max ulp: div %.2f sqrt %.2f rsqrt %.2f; exact: div %.3f sqrt %.3f rsqrt %.3f"
          % (e_div.max(), e_sq.max(), e_rsq.max(), (e_div == 0).mean(), (e_sq == 0).mean(),
             (e_rsq == 0).mean()), flush=True)
    assert e_div.max() <= 2.0
    assert e_sq.max() <= 1.0
    assert e_rsq.max() <= 2.0


def test_exact_cases_stay_exact():
    from paper_1102_5202_amd import grmhd
    k = np.arange(1.0, 4097.0)
    x = k * k
    out = grmhd.device_arith(torch.from_numpy(x).to(DEV), torch.from_numpy(k).to(DEV)).cpu().numpy()
    assert np.array_equal(out[0], k)                  # k^2 / k
    assert np.array_equal(out[1], k)                  # sqrt of a perfect square
    p = 4.0 ** np.arange(-20, 21)
    o2 = grmhd.device_arith(torch.from_numpy(p).to(DEV), torch.from_numpy(np.ones_like(p)).to(DEV)).cpu().numpy()
    assert np.array_equal(o2[0], p)                   # x / 1
    assert np.array_equal(o2[2], 1.0 / np.sqrt(p))    # 1/sqrt of a power of 4

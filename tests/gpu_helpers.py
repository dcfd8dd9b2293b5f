"""Shared helpers for the GPU parity tests (inputs from the workload generator, expected values
from the oracle, results from the HIP library through its C ABI)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2204_03139_amd as p  # raises if the HIP library is missing
    p.load()
    return p


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def assert_rel(got, exp, rtol, what=""):
    got = np.asarray(got, np.float64)
    exp = np.asarray(exp, np.float64)
    err = np.abs(got - exp)
    bound = rtol * np.abs(exp)
    bad = err > bound
    assert not bad.any(), f"{what}: {bad.sum()} values beyond {rtol} relative; worst " \
        f"{(err / np.maximum(np.abs(exp), 1e-300)).max():.3e}"


def assert_grad(got, exp, exp_abs, rtol=1e-5, what="grad"):
    """|g - g64| <= rtol * sum|contributions| per component (plus a tiny absolute floor)."""
    got = np.asarray(got, np.float64)
    err = np.abs(got - exp)
    bound = rtol * exp_abs + 1e-30
    bad = err > bound
    assert not bad.any(), f"{what}: {bad.sum()} components beyond bound; worst ratio " \
        f"{(err / bound).max():.3e}"

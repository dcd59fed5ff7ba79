"""tm_factor_solve_noalloc (static scratch, no allocation, no synchronisation) against tm_factor_solve
through the C ABI: two calls in a row, the second with a smaller problem, in both precisions, plain and
transposed, with the default guard and with every system sent to the partial-pivoting re-run; and the
rejection of a problem whose factors do not fit the scratch."""
import sys

import numpy as np
import pytest
import torch

import synth
from paper_1809_05608_amd import tm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("guard", ["default", "all"])
@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("precision", [tm.PREC_FP64, tm.PREC_MIXED])
def test_noalloc_solve_equals_factor_solve(monkeypatch, precision, transpose, guard):
    if guard == "all":
        monkeypatch.setenv("TM_GROWTH_LIMIT", "0")
    for shape in (dict(S=2, R=11, I=23, N=20), dict(S=1, R=5, I=17, N=13)):      # second call smaller
        say("case noalloc", precision, transpose, guard, shape)
        w = synth.make_custom(**shape)
        wd = w.to("cuda")
        ctx = tm.Context(tm.problem_of(wd, precision))
        f = tm.DeviceFields.of(wd)
        rng = np.random.default_rng(sum(shape.values()))
        psi = torch.as_tensor(w.psi_n.numpy() * 1.02, device="cuda")
        rhs = torch.as_tensor(rng.standard_normal(tuple(psi.shape)), device="cuda")
        ref = torch.empty_like(psi)
        ctx.factor_solve(f, psi, rhs, ref, transpose)
        x = torch.full_like(psi, float("nan"))
        flags = torch.full((w.S, w.R), -1, dtype=torch.int32, device="cuda")
        ctx.factor_solve_noalloc(f, psi, rhs, x, transpose, flags)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(x.cpu().numpy(), ref.cpu().numpy())
        fl = flags.cpu().numpy()
        assert not np.any(fl & tm.FLAG_ZERO_PIVOT)
        if guard == "all":
            assert np.all(fl == tm.FLAG_PIVOT_FALLBACK)
        else:
            assert np.all(fl == 0)
        ctx.close()


def test_noalloc_rejects_a_problem_beyond_the_scratch():
    """One system of 4000 zones x 32 groups: 16 factor slots of 33.8 MB exceed the 256 MiB scratch."""
    say("case noalloc too large")
    w = synth.make_custom(S=1, R=1, I=4000, N=32)
    wd = w.to("cuda")
    ctx = tm.Context(tm.problem_of(wd, tm.PREC_FP64))
    f = tm.DeviceFields.of(wd)
    x = torch.empty_like(wd.psi_n)
    with pytest.raises(tm.TMError) as e:
        ctx.factor_solve_noalloc(f, wd.psi_n, wd.psi_n, x, False)
    assert e.value.status == 6                      # TM_ERR_WORKSPACE
    ctx.close()

"""The reduction folded into the next pass-1 launch (three launches per Lanczos
half-step, ssa_opts.unfused = 0) against the fused four-launch half-step (unfused = 2).

Every pass-1 workgroup sums the partials of the last pass 3 in the reduction kernel's
order, so a folded solve gives the four-launch solve's bits.  A vector that needs a
DGKS pass or a fresh direction (breakdown, Sec. 3.2.2) cannot be finished inside the
pass-1 launch: the solve then restarts as four launches, with the same result as a
four-launch solve from the start."""
import sys

import numpy as np
import pytest

from paper_0911_4498_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ssa():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0911_4498_amd import ssa as mod
    mod.load()
    return mod


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def solve(ssa, f, L, k, **kw):
    plan = ssa.Plan(len(f), L, k, **kw)
    s, U, V, info = plan.truncated_svd(torch.tensor(f, device="cuda"), k)
    torch.cuda.synchronize()
    out = (s.cpu(), U.cpu(), V.cpu(), info)
    plan.close()
    return out


def same_bits(a, b):
    for x, y in zip(a[:3], b[:3]):
        assert x.shape == y.shape
        assert torch.equal(x.view(torch.int8) if x.dtype != torch.float64 else x.view(torch.int64),
                           y.view(torch.int8) if y.dtype != torch.float64 else y.view(torch.int64))
    assert a[3].steps == b[3].steps and a[3].steps_run == b[3].steps_run
    assert a[3].converged == b[3].converged


@pytest.mark.parametrize("N,L,k,reorth", [(1000, 500, 10, 0), (20000, 10000, 12, 0), (100000, 50000, 20, 0),
                                          (40000, 20000, 8, 1), (30001, 9000, 16, 0)])
def test_fold_same_bits_as_four_launches(ssa, N, L, k, reorth):
    say(f"fold vs four launches: N={N} L={L} k={k} reorth={reorth}")
    f = inputs.c2_series(N) if N >= 20000 else inputs.c1_series(N)
    a = solve(ssa, f, L, k, reorth=reorth)
    b = solve(ssa, f, L, k, reorth=reorth, unfused=2)
    say(f"  launches {a[3].half_step_launches}/{b[3].half_step_launches} steps {a[3].steps} "
        f"run {a[3].steps_run} dgks {a[3].dgks_passes} restarts {a[3].restarts}")
    assert a[3].half_step_launches == 3 and b[3].half_step_launches == 4
    same_bits(a, b)


def test_fold_many_columns_same_bits(ssa):
    """Past 160 columns the partials are summed by a launch of their own before pass 1
    (same order, same bits)."""
    f = inputs.c2_series(20000)
    # (one stopping test, at the step cap: the run takes all 240 steps)
    a = solve(ssa, f, 10000, 16, d_max=240, tol=1e-30, check_every=1000)
    b = solve(ssa, f, 10000, 16, d_max=240, tol=1e-30, check_every=1000, unfused=2)
    say(f"  steps {a[3].steps} run {a[3].steps_run} launches {a[3].half_step_launches}")
    assert a[3].half_step_launches == 3 and a[3].steps_run > 200
    same_bits(a, b)


@pytest.mark.parametrize("check_every", [1, 3])
def test_fold_same_bits_any_check_interval(ssa, check_every):
    """The stopping test of step j waits for the U half's first launch (it yields alpha_j);
    every check interval gives the four-launch bits."""
    f = inputs.c2_series(20000)
    a = solve(ssa, f, 10000, 8, check_every=check_every)
    b = solve(ssa, f, 10000, 8, check_every=check_every, unfused=2)
    assert a[3].half_step_launches == 3
    same_bits(a, b)


@pytest.mark.parametrize("N,L,k", [(2000, 1000, 4), (5000, 1200, 6)])
def test_breakdown_restarts_unfolded(ssa, N, L, k):
    """A rank-2 series: beta_3 vanishes, the folded solve asks for a fresh direction and
    starts over as four launches, with the four-launch result."""
    f = inputs.sinusoid(N, 37.0)
    say(f"breakdown: N={N} L={L} k={k}")
    a = solve(ssa, f, L, k)
    b = solve(ssa, f, L, k, unfused=2)
    say(f"  launches {a[3].half_step_launches} restarts {a[3].restarts} steps {a[3].steps}")
    assert b[3].restarts > 0
    assert a[3].half_step_launches == 4 and a[3].restarts == b[3].restarts
    same_bits(a, b)
    s = a[0].numpy()
    assert s[0] > 0 and s[1] > 0 and np.all(s[2:] < 1e-4 * s[0])


def test_plan_reuse_after_restart(ssa):
    """A plan whose solve restarted unfolded folds again on its next series."""
    f_bad = inputs.sinusoid(4000, 29.0)
    f_ok = inputs.c1_series(4000)
    plan = ssa.Plan(4000, 2000, 6)
    _, _, _, i1 = plan.truncated_svd(torch.tensor(f_bad, device="cuda"), 6)
    s2, U2, V2, i2 = plan.truncated_svd(torch.tensor(f_ok, device="cuda"), 6)
    torch.cuda.synchronize()
    assert i1.half_step_launches == 4 and i2.half_step_launches == 3
    b = solve(ssa, f_ok, 2000, 6, unfused=2)
    same_bits((s2.cpu(), U2.cpu(), V2.cpu(), i2), b)
    plan.close()


def test_many_workgroups_stay_four_launches(ssa):
    """Pass 3 with more than 256 workgroups (M/2 = 100000 splits as 250 x 400): the
    reduction stays a launch of its own."""
    f = inputs.c2_series(200000)
    plan = ssa.Plan(200000, 100000, 8)
    d = plan.desc
    s, U, V, info = plan.truncated_svd(torch.tensor(f, device="cuda"), 8)
    torch.cuda.synchronize()
    nblk = (d.M2 + d.cb - 1) // d.cb
    say(f"  M2={d.M2} cb={d.cb} launches={info.half_step_launches}")
    assert info.half_step_launches == (3 if nblk <= 256 else 4)
    plan.close()

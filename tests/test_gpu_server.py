"""Continuous batching (ssa_server_*): requests admitted at different ticks, fewer
slots than requests and a bounded pool give the same bits as the batch engine with
the same keys, agree with the FP64 oracle, and hand every pool byte back."""
import sys

import numpy as np
import pytest

from tests import parity
from tests.test_gpu_batch import compare_one, small_batch

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


def run_server(ssa, series, Ls, ks, keys, slots, pool_bytes, per_tick=1):
    srv = ssa.Server(n_max=1500, k_max=16, slots=slots, pool_bytes=pool_bytes)
    free0 = srv.status()["pool_free"]
    outs = {}
    pending = list(range(len(series)))
    done = {}
    ticks = 0
    while len(done) < len(series):
        for _ in range(per_tick):
            if pending:
                s = pending.pop(0)
                outs[s] = srv.submit(s, series[s], Ls[s], ks[s], key=keys[s])
        for rid, out in srv.step():
            done[rid] = out
        ticks += 1
        assert ticks < 20000
    st = srv.status()
    say(f"server: {len(series)} requests in {ticks} ticks, status {st}")
    assert st["queued"] == 0 and st["active"] == 0 and st["finalizing"] == 0
    assert st["pool_free"] == free0
    return done


def test_server_equals_batch_and_oracle(ssa):
    series, Ls, ks = small_batch(16)
    keys = [9000 + s for s in range(16)]
    say("batch engine reference: solving")
    b = ssa.Batch(n_max=1500, k_max=16, max_series=16)
    ref = b.solve(series, Ls, ks, keys=keys)
    torch.cuda.synchronize()
    # 5 slots and a pool that holds only a few regions at a time
    per = max(ssa.Server(n_max=1500, k_max=16, slots=1, pool_bytes=1 << 24).request_bytes(len(f), L, k)
              for f, L, k in zip(series, Ls, ks))
    say(f"largest request region {per} bytes")
    done = run_server(ssa, series, Ls, ks, keys, slots=5, pool_bytes=3 * per + (1 << 20))
    for s in range(16):
        out = done[s]
        for key in ("sigma", "U", "V", "recon"):
            a = out[key].cpu().numpy()
            r = ref[key][s].cpu().numpy()
            assert np.array_equal(a, r), (s, key)
        assert np.array_equal(out["info"].cpu().numpy(), ref["info"][s].cpu().numpy())
    for s in (0, 3, 9):
        f, L, k = series[s], Ls[s], ks[s]
        out = done[s]
        rep = compare_one(f, L, k, out["sigma"], out["U"], out["V"], out["recon"])
        say(f"request {s}: N={len(f)} L={L} k={k} {rep}")


def test_server_rejects_oversized_request(ssa):
    srv = ssa.Server(n_max=1500, k_max=16, slots=2, pool_bytes=1 << 20)
    f = np.sin(np.arange(1400) * 0.1)
    with pytest.raises(ssa.SsaError):
        srv.submit(0, f, 700, 16)  # region larger than the whole pool
    with pytest.raises(ssa.SsaError):
        srv.submit(1, np.zeros(3000), 1000, 8)  # longer than n_max


def run_mixed(ssa, reqs, long_slots, pool_bytes, slots=4):
    """Serve (rid, f, L, k, key) requests, all submitted at once, on a server whose batched
    engine takes N <= 1500; longer ones go to the long path."""
    srv = ssa.Server(n_max=1500, k_max=16, slots=slots, pool_bytes=pool_bytes, n_long_max=1 << 17,
                     long_slots=long_slots)
    free0 = srv.status()["pool_free"]
    for rid, f, L, k, key in reqs:
        srv.submit(rid, f, L, k, key=key)
    done, ticks = {}, 0
    while len(done) < len(reqs):
        for rid, out in srv.step():
            done[rid] = out
        ticks += 1
        assert ticks < 20000
    torch.cuda.synchronize()
    st = srv.status()
    say(f"mixed server: {len(reqs)} requests in {ticks} ticks, status {st}")
    assert st["queued"] == 0 and st["active"] == 0 and st["finalizing"] == 0 and st["pool_free"] == free0
    srv.close()
    return done


def test_long_request_same_bits_alone_and_in_the_mix(ssa):
    """A request above the batched engine's n_max runs the single-series solver on a plan
    bound to its pool region, advanced one check interval per tick.  It gives the same bits
    served alone and served beside another long request and batched ones (its key seeds its
    start vector), and agrees with the FP64 oracle."""
    from paper_0911_4498_amd import inputs
    fA, _, _ = inputs.c3_series(5, N=6000)
    fB, _, _ = inputs.c3_series(6, N=60000)
    series, Ls, ks = small_batch(6)
    say("long request alone")
    alone = run_mixed(ssa, [(0, fA, 3000, 12, 77)], long_slots=1, pool_bytes=1 << 30)[0]
    say("long request in the mix")
    mix = [(1, fB, 30000, 16, 78)] + [(10 + s, series[s], Ls[s], ks[s], 500 + s) for s in range(3)]
    mix += [(0, fA, 3000, 12, 77)] + [(10 + s, series[s], Ls[s], ks[s], 500 + s) for s in range(3, 6)]
    done = run_mixed(ssa, mix, long_slots=2, pool_bytes=1 << 30)
    for key in ("sigma", "U", "V", "recon", "info"):
        assert np.array_equal(done[0][key].cpu().numpy(), alone[key].cpu().numpy()), key
    info = alone["info"].cpu().numpy()
    say(f"long request: info {info}")
    assert info[1] == 1
    rep = compare_one(fA, 3000, 12, alone["sigma"], alone["U"], alone["V"], alone["recon"], dense=False)
    say(f"long request against the oracle: {rep}")
    assert done[1]["info"].cpu().numpy()[1] == 1

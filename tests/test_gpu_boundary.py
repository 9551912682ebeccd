"""GPU tests of the C ABI contract: a simulation busy on one stream refuses
steps enqueued on another (SDM_EAGAIN) and enqueues nothing; set-up calls
synchronise their own stream only."""
import numpy as np
import pytest

from paper_2103_17238_amd import inputs as I

from sdm_testutil import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_17238_amd import binding

    return binding


def _spin(stream, cycles=50_000_000):
    """A bounded spin kernel on `stream` (torch's own), so that work enqueued
    after it is still pending for a while."""
    import torch

    with torch.cuda.stream(stream):
        torch.cuda._sleep(cycles)


def test_eagain_when_member_busy_on_another_stream(B):
    import torch

    st = I.random_cells(48, 300, n_attr=1, rng_seed=11, p_boost=20.0)
    sim = B.Sim(st)
    ref = B.Sim(st)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ws = B.workspace_tensor(B.sdm_batch_workspace_bytes([sim.handle]))
    batch = B.sdm_batch_create([sim.handle], ws, s2)
    torch.cuda.synchronize()

    say("eagain: step on s1 behind a spin, then batch step on s2")
    _spin(s1)
    B.sdm_coalescence_step(sim.handle, 1, s1)
    with pytest.raises(B.SdmError) as e:
        B.sdm_batch_step(batch, 1, s2)
    assert e.value.status == B.SDM_EAGAIN
    assert B.sdm_get_step(sim.handle) == 1  # nothing was enqueued
    with pytest.raises(B.SdmError) as e:  # a solo step on s2 likewise
        B.sdm_coalescence_step(sim.handle, 1, s2)
    assert e.value.status == B.SDM_EAGAIN
    B.sdm_coalescence_step(sim.handle, 1, s1)  # the same stream is fine
    s1.synchronize()
    B.sdm_batch_step(batch, 2, s2)  # idle now: accepted on s2
    say("eagain: batch busy on s2, solo step on s1")
    _spin(s2)
    B.sdm_batch_step(batch, 1, s2)
    with pytest.raises(B.SdmError) as e:
        B.sdm_coalescence_step(sim.handle, 1, s1)
    assert e.value.status == B.SDM_EAGAIN
    s2.synchronize()
    assert B.sdm_get_step(sim.handle) == 5

    ref.step(5)
    xa, va, aa = sim.state()
    xb, vb, ab = ref.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(aa, ab)
    B.sdm_batch_free(batch)
    sim.close()
    ref.close()


def test_init_does_not_wait_for_other_streams(B):
    """sdm_init on one stream returns while a long spin runs on another."""
    import time

    import torch

    busy, side = torch.cuda.Stream(), torch.cuda.Stream()
    st = I.random_cells(8, 100, rng_seed=5)
    torch.cuda.synchronize()
    _spin(busy, 400_000_000)
    ev = torch.cuda.Event()
    ev.record(busy)
    t0 = time.perf_counter()
    with torch.cuda.stream(side):
        sim = B.Sim(st, stream=side)
    dt_init = time.perf_counter() - t0
    still_busy = not ev.query()
    busy.synchronize()
    dt_all = time.perf_counter() - t0
    say(f"init {dt_init * 1e3:.2f} ms while the spin ran {dt_all * 1e3:.2f} ms; "
        f"spin still running at return: {still_busy}")
    assert still_busy, "sdm_init waited for work on another stream"
    sim.close()

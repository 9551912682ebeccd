"""GPU tests of the C ABI contract: a simulation busy on one stream refuses
steps enqueued on another (SDM_EAGAIN) and enqueues nothing; set-up calls
synchronise their own stream only."""
import os

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


def _spin(stream, cycles=100_000_000):
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
    # the first step of each plan creates its side stream and events: done
    # here, outside the timed windows below
    B.sdm_coalescence_step(sim.handle, 1, s1)
    s1.synchronize()
    B.sdm_batch_step(batch, 1, s2)
    s2.synchronize()

    say("eagain: step on s1 behind a spin, then batch step on s2")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s1)
    _spin(s1)
    e1.record(s1)
    B.sdm_coalescence_step(sim.handle, 1, s1)
    busy = None
    try:
        B.sdm_batch_step(batch, 1, s2)
    except B.SdmError as e:
        busy = e.status
    s1.synchronize()
    say(f"  spin {e0.elapsed_time(e1):.1f} ms; batch step on s2 returned {busy}")
    assert busy == B.SDM_EAGAIN
    assert B.sdm_get_step(sim.handle) == 3  # nothing was enqueued
    _spin(s1)
    B.sdm_coalescence_step(sim.handle, 1, s1)
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
    assert B.sdm_get_step(sim.handle) == 8

    ref.step(8)
    xa, va, aa = sim.state()
    xb, vb, ab = ref.state()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb) and np.array_equal(aa, ab)
    B.sdm_batch_free(batch)
    sim.close()
    ref.close()


def test_init_does_not_wait_for_other_streams(B):
    """sdm_init synchronises its own stream only: checked in a fresh process
    (tests/gpu_init_nowait.py), where the stream under test and the busy one
    cannot share a hardware queue."""
    import subprocess
    import sys

    say("init-does-not-wait check in a fresh process")
    here = os.path.dirname(os.path.abspath(__file__))
    r = subprocess.run([sys.executable, os.path.join(here, "gpu_init_nowait.py")],
                       capture_output=True, text=True, timeout=180)
    say(r.stdout.strip())
    if r.returncode != 0:
        say(r.stderr[-2000:])
    assert r.returncode == 0, "sdm_init waited for work on another stream"

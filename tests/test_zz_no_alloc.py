"""The allocation-free displacement entry point (sdm_displace_noalloc, whose
workspace is a file-scope device array of the library) against the entry
point with a caller workspace (sdm_displace), through the C ABI: every output
bit-exact on two calls in a row, the second with a smaller domain (so the
second call reuses scratch the first one filled), and a domain above the
scratch limit refused on the host with nothing enqueued."""
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


def _case(nx, nz, max_sd, n_attr, seed):
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, max_sd + 1, size=nx * nz)
    off = np.zeros(nx * nz + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    n = int(off[-1])
    xi = rng.integers(0, 10 ** 9, size=n).astype(np.int64)
    v = rng.random(n)
    attrs = rng.random((n_attr, n))
    cx, cz = I.random_courant(nx, nz, 0.9, seed=seed + 100)
    pos = I.positions(n, seed=seed + 200)
    return cx, cz, xi, v, attrs, pos, off


def _outputs(n, nx, nz, A):
    import torch

    return [torch.full((n,), -5, dtype=torch.int64, device="cuda"),
            torch.full((n,), -5.0, dtype=torch.float64, device="cuda"),
            torch.full((A, n), -5.0, dtype=torch.float64, device="cuda") if A else None,
            torch.full((2, n), -5.0, dtype=torch.float64, device="cuda"),
            torch.full((nx * nz + 1,), -5, dtype=torch.int64, device="cuda")]


def _host(ts, n):
    return [t.cpu().numpy() if t is not None else np.zeros((0, n)) for t in ts]


def test_noalloc_equals_workspace_entry_point(B):
    import torch

    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    for nx, nz, max_sd, A, seed in [(64, 48, 90, 6, 1), (20, 10, 300, 2, 2)]:
        say(f"noalloc displacement nx={nx} nz={nz} max_sd={max_sd} A={A}")
        cx, cz, xi, v, attrs, pos, off = _case(nx, nz, max_sd, A, seed)
        n = xi.size
        ins = [d(xi), d(v), d(attrs) if A else None, d(pos), d(off)]
        ref = _outputs(n, nx, nz, A)
        got = _outputs(n, nx, nz, A)
        st_ref = torch.zeros(1, dtype=torch.int32, device="cuda")
        st_got = torch.zeros(1, dtype=torch.int32, device="cuda")
        ws = B.workspace_tensor(B.sdm_displace_workspace_bytes(nx, nz))
        B.sdm_displace(nx, nz, d(cx), d(cz), *ins, *ref, st_ref, ws)
        B.sdm_displace_noalloc(nx, nz, d(cx), d(cz), *ins, *got, st_got)
        torch.cuda.synchronize()
        for g, r, nm in zip(_host(got, n), _host(ref, n), ("xi", "v", "attrs", "pos", "off")):
            assert np.array_equal(g, r), nm
        assert int(st_got.item()) == int(st_ref.item()) == 0


def test_noalloc_refuses_domains_above_the_scratch(B):
    """Host-side check: nothing is launched (the fake pointers are never read)."""
    import torch

    lim = B.sdm_displace_noalloc_max_cells()
    assert lim == 2 ** 17
    nx, nz = 512, 512  # 2^18 cells
    assert nx * nz > lim
    one = torch.zeros(8, dtype=torch.float64, device="cuda")
    off = torch.zeros(nx * nz + 1, dtype=torch.int64, device="cuda")
    off2 = torch.zeros(nx * nz + 1, dtype=torch.int64, device="cuda")
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    ev = torch.empty(0, dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(B.SdmError) as err:
        B.sdm_displace_noalloc(nx, nz, one, one, e, ev, None, ev, off, e, ev, None, ev, off2,
                               status)
    assert err.value.status == B.SDM_ENOMEM
    torch.cuda.synchronize()
    assert int(status.item()) == 0

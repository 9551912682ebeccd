"""Pins of the oracle's random numbers and permutation (CPU only).

- Philox4x32-10 against rocRAND's engine, a separately written implementation
  of the same published generator (Salmon et al. 2011).
- The per-cell permutation against Python's own sort of (key, slot) tuples
  built from those pinned generator words.
- Uniformity of the permutation over all n! orders (chi-square).
"""
import itertools
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_ref():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("hipcc / rocRAND headers not available")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "rocrand_philox_ref")
    subprocess.check_call([hipcc, "-O1", "--offload-host-only", "-o", exe,
                           os.path.join(HERE, "rocrand_philox_ref.cpp")], cwd=d)

    def run(n, c0, c1, c2, c3, seed):
        out = subprocess.check_output([exe, str(n), str(c0), str(c1), str(c2), str(c3),
                                       str(seed)], text=True)
        return np.array([[int(w) for w in ln.split()] for ln in out.strip().splitlines()],
                        dtype=np.uint64).astype(np.uint32)

    yield run
    shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("c0,c1,c2,c3,seed", [
    (0, 0, 0, 0, 0),
    (0, 7, 123, 2, 0),
    (0xFFFFFF00, 1, 0xFFFFFFFF, 5, 0x123456789ABCDEF0),
    (1000, 65535, 3599, 1, 42),
    (12345, 4095, 199, 9, 0xFFFFFFFFFFFFFFFF),
])
def test_philox_matches_rocrand(orc, rocrand_ref, c0, c1, c2, c3, seed):
    n = 3000
    ours = orc.philox_fill(c0, c1, c2, c3, seed, n)
    ref = rocrand_ref(n, c0, c1, c2, c3, seed)
    assert ours.shape == ref.shape
    assert np.array_equal(ours, ref)


def test_phi_exact_values(orc):
    assert orc.phi_from_words(0, 0) == 0.0
    assert orc.phi_from_words(0, 1 << 11) == 2.0 ** -53
    assert orc.phi_from_words(0, (1 << 11) - 1) == 0.0  # low 11 bits dropped
    top = orc.phi_from_words(0xFFFFFFFF, 0xFFFFFFFF)
    assert top == 1.0 - 2.0 ** -53 and top < 1.0
    assert orc.phi_from_words(0x80000000, 0) == 0.5


def _keys_from_pinned_words(orc, n_slots, seed, c, s, u):
    words = orc.philox_fill(0, c, s, 2 * u, seed, (n_slots + 3) // 4)
    return [int(words[j // 4, j % 4]) for j in range(n_slots)]


@pytest.mark.parametrize("n_slots,c,s,u,seed", [
    (1, 0, 0, 0, 0), (2, 3, 1, 0, 7), (7, 11, 5, 0, 1), (64, 0, 0, 0, 0),
    (513, 17, 999, 0, 3), (4096, 2, 3599, 2, 0xDEADBEEF), (8192, 0, 0, 1, 0),
])
def test_cell_order_is_key_slot_sort(orc, n_slots, c, s, u, seed):
    rng = np.random.default_rng(n_slots)
    xi = rng.integers(1, 100, size=n_slots).astype(np.int64)
    xi[rng.random(n_slots) < 0.25] = 0  # dead slots are left out
    keys = _keys_from_pinned_words(orc, n_slots, seed, c, s, u)
    expect = [j for _, j in sorted((keys[j], j) for j in range(n_slots) if xi[j] > 0)]
    got = orc.cell_order(xi, seed, c, s, u)
    assert got.tolist() == expect


def test_cell_order_tie_broken_by_slot(orc):
    # With 2^17 slots some 32-bit keys collide; the order must still be (key, slot).
    n = 1 << 17
    xi = np.ones(n, dtype=np.int64)
    keys = np.array(_keys_from_pinned_words(orc, n, 5, 1, 2, 0), dtype=np.int64)
    got = orc.cell_order(xi, 5, 1, 2, 0)
    expect = np.lexsort((np.arange(n), keys))
    assert np.array_equal(got, expect)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_permutation_uniform(orc, n):
    draws = 24000 if n <= 4 else 60000
    counts = {}
    xi = np.ones(n, dtype=np.int64)
    for s in range(draws):
        perm = tuple(orc.cell_order(xi, 11, s % 97, s // 97, 0).tolist())
        counts[perm] = counts.get(perm, 0) + 1
    perms = list(itertools.permutations(range(n)))
    assert set(counts) <= set(perms)
    obs = np.array([counts.get(p, 0) for p in perms], dtype=np.float64)
    exp = np.full(len(perms), draws / math.factorial(n))
    pval = stats.chisquare(obs, exp).pvalue
    assert pval > 1e-3, (obs, pval)

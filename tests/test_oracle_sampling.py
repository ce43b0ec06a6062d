"""Pins of the oracle's sampling operators and index generators (CPU only)."""

import json
import os

import numpy as np
import pytest
import scipy.linalg

from oracle.sampling import (Sampling, apply_c, apply_ct, fisher_yates, fwht,
                             rsp_mask, shd_pattern, splitmix64_stream)
from oracle.dense import dense_sampling_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_vector():
    ref = json.load(open(os.path.join(GOLDEN, "splitmix64_seed1234567.json")))
    gen = splitmix64_stream(ref["seed"])
    assert [next(gen) for _ in range(5)] == [int(v) for v in ref["outputs"]]


@pytest.mark.parametrize("n,seed", [(1, 0), (7, 3), (1024, 2), (16384, 9)])
def test_fisher_yates_is_permutation(n, seed):
    a = fisher_yates(n, seed)
    assert sorted(a) == list(range(n))


def test_fisher_yates_uniform_on_small_set():
    """All 6 orderings of 3 items appear with roughly equal frequency."""
    counts = {}
    for seed in range(6000):
        key = tuple(fisher_yates(3, seed))
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 6
    assert all(800 < c < 1200 for c in counts.values())


@pytest.mark.parametrize("n_pix,mc,seed", [(1024, 256, 2), (16384, 2048, 2), (16, 16, 1)])
def test_rsp_mask_sorted_unique(n_pix, mc, seed):
    idx = rsp_mask(n_pix, mc, seed)
    assert idx.dtype == np.int32 and len(idx) == mc
    assert np.all(np.diff(idx) > 0) and idx[0] >= 0 and idx[-1] < n_pix


def test_shd_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        shd_pattern(96 * 96, 100, 1)


@pytest.mark.parametrize("n", [64, 1024])
def test_fwht_matches_sylvester_matrix(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, n))
    W = scipy.linalg.hadamard(n).astype(np.float64)
    assert np.allclose(fwht(x), x @ W.T, rtol=0, atol=1e-10)


@pytest.mark.parametrize("kind", ["full", "points", "hadamard"])
def test_c_ct_identity_and_transpose(kind):
    n_pix, nt = 64, 5
    smp = {"full": Sampling.full(n_pix), "points": Sampling.points(n_pix, 16, 3),
           "hadamard": Sampling.hadamard(n_pix, 8, 4)}[kind]
    Cm = dense_sampling_matrix(smp, n_pix)
    assert np.allclose(Cm @ Cm.T, np.eye(smp.mc), atol=1e-13)        # C C^T = I
    rng = np.random.default_rng(1)
    s = rng.standard_normal((nt, 8, 8))
    f = apply_c(s, smp)
    assert np.allclose(f, s.reshape(nt, -1) @ Cm.T, atol=1e-13)
    r = rng.standard_normal((nt, smp.mc))
    assert np.allclose(apply_ct(r, smp, 8, 8).reshape(nt, -1), r @ Cm, atol=1e-13)


def test_hadamard_entries_are_pm_one_over_sqrt_n():
    n_pix = 256
    smp = Sampling.hadamard(n_pix, 32, 4)
    Cm = dense_sampling_matrix(smp, n_pix)
    assert np.allclose(np.abs(Cm) * np.sqrt(n_pix), 1.0)

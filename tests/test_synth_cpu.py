"""Host checks of the seeded input generators (no device): the shapes and
structure the benchmark workloads rely on."""
import numpy as np

from paper_2606_06811_amd import synth


def _strand_free_counts(codes):
    c = np.bincount(codes, minlength=4)
    return c[0] + c[3], c[1] + c[2]            # A+T, C+G: unchanged by reverse complements


def test_many_svs_moves_bases_without_losing_any():
    rng = synth.rng_for(11)
    codes = synth.iid_codes(rng, 200_000)
    soft = np.zeros(codes.shape[0], bool)
    soft[1000:3000] = True
    c, s = synth.many_svs(synth.rng_for(12), codes, soft, 5, 5, 2000)
    assert c.shape == codes.shape and s.shape == soft.shape
    assert _strand_free_counts(c) == _strand_free_counts(codes)
    assert int(s.sum()) == int(soft.sum())
    assert not np.array_equal(c, codes)
    # deterministic for a seed
    c2, _ = synth.many_svs(synth.rng_for(12), codes, soft, 5, 5, 2000)
    assert np.array_equal(c, c2)


def test_segmental_duplications_copy_target_segments():
    rng = synth.rng_for(13)
    n = 400_000
    codes = synth.iid_codes(rng, n)
    soft = np.zeros(n, bool)
    before = codes.copy()
    c, _ = synth.segmental_duplications(synth.rng_for(14), codes, soft, 0.05, 1000, 5000, 0.0, 0.0)
    assert c.shape[0] == n
    changed = int((c != before).sum())
    # at least 5 % of the sequence was overwritten by copies, and exact copies (divergence 0)
    # make some 64-mer occur twice
    assert changed > 0.02 * n
    k = 64
    words = {c[p:p + k].tobytes() for p in range(0, n - k)}
    assert len(words) < n - k                   # a repeated 64-mer exists
    assert len({before[p:p + k].tobytes() for p in range(0, n - k)}) == n - k   # none before


def test_pair_segdup_small_shapes():
    T, Q = synth.pair_segdup(n=2_000_000, sd_lo=1000, sd_hi=20_000)
    assert T.shape[0] == 2_000_000 and len(Q) == 1
    assert abs(Q[0].shape[0] - T.shape[0]) < 0.01 * T.shape[0]     # indels change the length a little
    assert set(np.unique(T).tolist()) <= set(b"ACGTacgt")

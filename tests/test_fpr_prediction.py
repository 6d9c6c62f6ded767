"""The false-positive prediction used for the FPR-vs-size curve, pinned on the
CPU: for k-mers absent from the filter whose shard is uniform over the shards
and whose k-s+1 s-mers hash independently (Eq. 1 per sector, Eq. 2 across
s-mers), the chance that all (k-s+1)*H bits are set is, averaged over shards,
the product over sectors c of p_c^((k-s+1) n_c), where p_c is the set-bit
fraction of the shard's words of sector c (a hash index's word is uniform among
its sector's S/4 words) and n_c the hash indices t < H with t mod 4 = c.

The oracle inserts a genome-like sequence (GC 41%) and answers independent
uniform random 31-mers (each followed by an 'N', so each is its own record);
the number answered present must lie in the 99.9% Poisson interval of
n times the prediction (a sum of independent Bernoulli trials with unequal
rates varies less than a Poisson count of the same mean, so the interval is
conservative).  A GPU test checks the library's sbf_estimate_fpr against the
same formula on the GPU's own bits."""

import numpy as np
import pytest
from scipy.stats import poisson

import oracle
import synth


def predicted_fpr(F: np.ndarray, k: int, s: int, H: int, S: int) -> float:
    words = F.reshape(-1, S)
    z1 = k - s + 1
    prob = np.ones(words.shape[0])
    for c in range(4):
        n_c = len([t for t in range(H) if t % 4 == c])
        cols = [c + 4 * g for g in range(S // 4)]
        p_c = np.bitwise_count(words[:, cols]).sum(axis=1) / (64.0 * len(cols))
        prob *= p_c ** (z1 * n_c)
    return float(prob.mean())


@pytest.mark.parametrize("S,bits,H", [(4, 1 << 22, 4), (16, 1 << 22, 4), (8, 1 << 23, 8), (4, 1 << 21, 2)])
def test_uniform_kmer_fpr_matches_prediction(S, bits, H):
    k, s, m = 31, 28, 16
    p = oracle.Params(k, s, m, H, bits, shard_words=S)
    g = synth.background(1_000_000, 41)
    F = oracle.insert(p, p.empty(), g)
    n = 400_000
    q = synth.separated_uniform_kmers(n, k, 43).numpy()
    present = int(oracle.query(p, F, q).sum())
    mu = n * predicted_fpr(F, k, s, H, S)
    lo, hi = poisson.ppf(0.0005, mu), poisson.ppf(0.9995, mu)
    print("S=%d bits=%d H=%d: %d present, expected %.1f [%d, %d]" % (S, bits, H, present, mu, lo, hi))
    assert mu > 20  # the test has statistical power
    assert lo <= present <= hi


def test_prediction_of_special_filters():
    """Empty filter: 0; full filter: 1; one sector half full, others full:
    exactly 0.5^((k-s+1) n_c) of that sector."""
    k, s, H, S = 31, 28, 4, 4
    F = np.zeros(64 * S, dtype=np.uint64)
    assert predicted_fpr(F, k, s, H, S) == 0.0
    F[:] = np.iinfo(np.uint64).max
    assert predicted_fpr(F, k, s, H, S) == 1.0
    F.reshape(-1, S)[:, 2] = np.uint64(0x00000000FFFFFFFF)
    assert predicted_fpr(F, k, s, H, S) == pytest.approx(0.5 ** 4)


@pytest.mark.gpu
@pytest.mark.parametrize("S,H", [(4, 4), (8, 4), (16, 8), (4, 3)])
def test_library_estimate_matches_formula(S, H):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_24417_amd import Filter

    g = synth.background(2_000_000, 44)
    f = Filter(31, 28, 16, H, 1 << 22, shard_words=S)
    f.insert(torch.from_numpy(g).cuda())
    est, set_bits = f.estimate_fpr()
    bits = f.get_bits()
    f.close()
    assert set_bits == int(np.bitwise_count(bits).sum())
    assert est == pytest.approx(predicted_fpr(bits, 31, 28, H, S), rel=1e-9)

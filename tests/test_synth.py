"""The seeded generators: determinism, counter addressing and the recipe's statistics."""
import numpy as np
import pytest

from paper_1302_4332_amd import synth


def test_chunk_addressing_is_block_independent():
    a = synth.genotypes_u8(64, 0, 3000, seed=7)
    b = synth.genotypes_u8(64, 1000, 2100, seed=7)
    assert np.array_equal(a[1000:2100], b)
    assert set(np.unique(a)) <= {0, 1, 2}


def test_genotype_float_matches_u8():
    assert np.array_equal(synth.genotypes(32, 5, 90, 3), synth.genotypes_u8(32, 5, 90, 3).astype(np.float64))


def test_allele_frequencies_in_range():
    g = synth.genotypes_u8(4000, 0, 512, seed=9).astype(float)
    f = g.mean(axis=1) / 2
    assert f.min() > 0.03 and f.max() < 0.52


def test_kinship_spd_and_mean_diagonal():
    Phi = synth.kinship(300, seed=1)
    assert np.array_equal(Phi, Phi.T)
    assert abs(np.mean(np.diag(Phi)) - (1 + 1e-3)) < 1e-9      # trace(G G^T)/2000 = n for standardised G
    assert np.linalg.eigvalsh(Phi).min() > 0.5e-3


def test_study_deterministic_and_causal():
    s1 = synth.make_study("c1_n10k_m100k", n=200, m=5000)
    s2 = synth.make_study("c1_n10k_m100k", n=200, m=5000)
    assert np.array_equal(s1.Phi, s2.Phi) and np.array_equal(s1.y, s2.y) and s1.causal == s2.causal
    assert 0 <= s1.causal < 5000
    XL = s1.XL
    assert np.all(XL[:, 0] == 1) and set(np.unique(XL[:, 1])) <= {0.0, 1.0}
    assert 40 < XL[:, 2].mean() < 60


def test_pack_dosages_2bit_layout():
    # sample k in bits [2 (k % 4), 2 (k % 4) + 2) of byte k // 4, pad bits zero
    g = np.array([[0, 1, 2, 3, 2], [3, 3, 3, 3, 0]], dtype=np.uint8)
    assert synth.pack_dosages_2bit(g).tolist() == [[0b11100100, 0b00000010], [0xFF, 0x00]]
    with pytest.raises(ValueError):
        synth.pack_dosages_2bit(np.array([[4]], dtype=np.uint8))


@pytest.mark.parametrize("n", [1, 4, 7, 330])
def test_pack_dosages_2bit_round_trip(n):
    g = np.random.default_rng(n).integers(0, 4, size=(9, n)).astype(np.uint8)
    P = synth.pack_dosages_2bit(g)
    assert P.shape == (9, (n + 3) // 4)
    back = np.stack([(P[:, k // 4] >> (2 * (k % 4))) & 3 for k in range(n)], axis=1)
    assert np.array_equal(back, g)


def test_imputed_dosages():
    """Non-integer SNP values: jitter within half a dosage of the genotype and
    independent of the block split; standardized columns have mean 0 and s.d. 1."""
    g = synth.genotypes(97, 1000, 1100, 5)
    j = synth.imputed_dosages(97, 1000, 1100, 5)
    assert j.shape == g.shape and np.all(np.abs(j - g) <= 0.5)
    assert np.mean(j != np.round(j)) > 0.99
    parts = np.concatenate([synth.imputed_dosages(97, 1000, 1030, 5), synth.imputed_dosages(97, 1030, 1100, 5)])
    assert np.array_equal(parts, j)
    s = synth.imputed_dosages(97, 0, 40, 5, "standardized")
    assert np.allclose(s.mean(axis=1), 0.0, atol=1e-12) and np.allclose(s.std(axis=1), 1.0)

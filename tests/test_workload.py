"""The seeded input generators: shapes, distributions and determinism."""
import numpy as np

from paper_1404_0424_amd import workload as W


def test_seeded_and_deterministic():
    a = W.uplink_frame(W.rng_for(3, 0), 4, 16, 4, 2, 6, 15.0)
    b = W.uplink_frame(W.rng_for(3, 0), 4, 16, 4, 2, 6, 15.0)
    assert np.array_equal(a.Y, b.Y) and np.array_equal(a.bits, b.bits)
    c = W.uplink_frame(W.rng_for(3, 1), 4, 16, 4, 2, 6, 15.0)
    assert not np.array_equal(a.H, c.H)


def test_iid_channel_variance():
    H = W.iid_channel(np.random.default_rng(0), 400, 64, 8)
    np.testing.assert_allclose(np.mean(np.abs(H) ** 2) * 64, 1.0, rtol=0.02)
    assert abs(np.mean(H)) < 0.01


def test_kronecker_channel_correlation():
    B, U = 16, 4
    H = W.kronecker_channel(np.random.default_rng(1), 40000, B, U, 0.5, 0.2)
    RB = np.einsum("nbu,ncu->bc", H, H.conj()) / (40000 * U)
    RU = np.einsum("nbu,nbv->uv", H.conj(), H) / (40000 * B)
    np.testing.assert_allclose(RB * B, W.exp_corr(B, 0.5), atol=0.03)
    np.testing.assert_allclose(RU * B / np.trace(RU * B) * U, W.exp_corr(U, 0.2), atol=0.03)


def test_qam_energy_and_noise_level():
    rng = np.random.default_rng(2)
    for m in (2, 4, 6, 8):
        x = W.qam_map(W.random_bits(rng, (20000,), m), m, 1.0)
        np.testing.assert_allclose(np.mean(np.abs(x) ** 2), 1.0, rtol=0.03)
    n = W.awgn(rng, (200000,), 0.3)
    np.testing.assert_allclose(np.mean(np.abs(n) ** 2), 0.3, rtol=0.01)
    assert W.n0_from_snr_db(10.0, 8, 32) == 0.8            # U*E_s/SNR
    assert W.n0_from_snr_db(10.0, 8, 32, definition="per_user") == 0.1


def test_uplink_model_holds():
    f = W.uplink_frame(np.random.default_rng(3), 3, 8, 2, 4, 4, 300.0)
    np.testing.assert_allclose(f.Y, f.H @ f.X, atol=1e-13)

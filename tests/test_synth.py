"""Host-side checks of the seeded input generator (CPU only)."""
import numpy as np

import synth


def test_bf16_round_known_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -3.0 - 2 ** -7, 2.0 ** -130, 0.0,
                  1.0 + 2 ** -8 + 2 ** -30, 3.5 * 2 ** -133, 2.5 * 2 ** -133])
    r = synth.bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa wins -> 1
    # 1 + 3*2^-8 is a tie between 1+2^-7 and 1+2^-6: even -> 1 + 2^-6
    exp = np.array([1.0, 1.0, 1.0 + 2 ** -6, 1.0, -3.0, 2.0 ** -130, 0.0, 1.0 + 2 ** -7, 4.0 * 2 ** -133, 2.0 * 2 ** -133])
    assert np.array_equal(r, exp)
    bits = synth.f64_to_bf16_bits(np.array([1.0, -2.0, 0.5]))
    assert list(bits) == [0x3F80, 0xC000, 0x3F00]
    assert np.array_equal(synth.bf16_bits_to_f64(bits), [1.0, -2.0, 0.5])


def test_bf16_round_matches_float32_route_away_from_ties():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(10000)
    # float32 has 24 bits: rounding a float64 that is not near a bf16 tie through float32 agrees
    r32 = x.astype(np.float32)
    u = r32.view(np.uint32).astype(np.uint64)
    low = u & 0xFFFF
    safe = (low != 0x8000)
    rounded = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    via32 = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    assert np.array_equal(synth.bf16_round(x)[safe], via32[safe])


def test_irwin_hall_moments_and_determinism():
    key = synth.stream_key(123, 0)
    g = synth.ih12(key, np.arange(200000))
    assert abs(g.mean()) < 0.01 and abs(g.var() - 1.0) < 0.02 and np.max(np.abs(g)) <= 6.0
    assert np.array_equal(g[:100], synth.ih12(key, np.arange(100)))
    g2 = synth.ih12(synth.stream_key(123, 1), np.arange(1000))
    assert abs(np.corrcoef(g[:1000], g2)[0, 1]) < 0.1


def test_b_is_symmetric_and_decays():
    key = synth.stream_key(5, 0)
    B = synth.b_chunk(key, 30, 40, 0, 40, "bf16")
    assert np.array_equal(B, B.transpose(0, 2, 1))
    assert np.array_equal(B, synth.bf16_round(B))
    band0 = np.mean(B[:, np.arange(30), np.arange(30)] ** 2)
    band12 = np.mean(B[:, np.arange(18), np.arange(12, 30)] ** 2)
    assert abs(band12 / band0 - np.exp(-4.0)) < 0.3 * np.exp(-4.0)
    # rows are independent of how they are chunked
    assert np.array_equal(B[7:9], synth.b_chunk(key, 30, 40, 7, 9, "bf16"))


def test_workload_shapes():
    inst = synth.workload("c1_eri24")
    assert inst.ERI.shape == (24,) * 4 and inst.B.shape == (96, 24, 24)
    assert np.max(np.abs(inst.C.T @ inst.C - np.eye(24))) < 1e-13
    assert np.all(np.diag(inst.H) <= -5) and np.all(np.diag(inst.H) >= -20)
    assert np.array_equal(inst.H, inst.H.T) and inst.gamma.shape == (10,)
    pes = synth.pes_scan(6, with_b=False)
    for p in pes:
        assert 40 <= p.wl.nbf <= 300 and p.wl.naux == 4 * p.wl.nbf and p.wl.npairs == p.wl.nbf // 10

"""Pins of the frequency-scheduling oracle (oracle/freq64.py): closed forms of
the frequency significance X (constant image, single pixel, pure cosine), a
brute-force O(N^2) DFT, invariance under circular shifts, the box
downsampling by its definition, and hand-built schedules."""
import math

import numpy as np
import pytest

from oracle.freq64 import TAU_F, downsample, next_levels, ratios, sample_frames, significance


def test_constant_image_has_only_the_dc_bin():
    H, W = 9, 14
    c = np.array([0.25, 0.5, 0.75])
    img = np.broadcast_to(c[:, None, None], (3, H, W))
    assert abs(significance(img) - H * W * math.sqrt((c ** 2).sum())) <= 1e-12 * H * W


def test_single_pixel_has_flat_spectrum():
    """A delta of values (a, b, c) has |F_ch| equal to the value at every bin."""
    H, W = 12, 10
    img = np.zeros((3, H, W))
    img[:, 5, 7] = (0.5, -2.0, 1.0)
    assert abs(significance(img) - H * W * math.sqrt(0.25 + 4.0 + 1.0)) <= 1e-12 * H * W


def test_pure_cosine_has_two_bins():
    H, W = 16, 20
    y, x = np.mgrid[0:H, 0:W]
    img = np.zeros((3, H, W))
    img[1] = np.cos(2 * np.pi * (3 * x / W + 5 * y / H))
    # two bins of magnitude H W / 2
    assert abs(significance(img) - H * W) <= 1e-9 * H * W


def _brute_dft(ch):
    H, W = ch.shape
    F = np.zeros((H, W), complex)
    for k in range(H):
        for l in range(W):
            s = 0j
            for y in range(H):
                for x in range(W):
                    s += ch[y, x] * np.exp(-2j * np.pi * (k * y / H + l * x / W))
            F[k, l] = s
    return F


@pytest.mark.parametrize("shape", [(4, 6), (5, 7), (3, 8)])
def test_significance_equals_brute_force_dft(shape):
    rng = np.random.default_rng(sum(shape))
    img = rng.uniform(0, 1, (3,) + shape)
    F = np.stack([_brute_dft(img[c]) for c in range(3)])
    want = np.sqrt((np.abs(F) ** 2).sum(axis=0)).sum()
    assert abs(significance(img) - want) <= 1e-12 * want


def test_significance_is_invariant_under_circular_shifts():
    rng = np.random.default_rng(5)
    img = rng.uniform(0, 1, (3, 30, 45))
    a = significance(img)
    b = significance(np.roll(img, (7, -11), axis=(1, 2)))
    assert abs(a - b) <= 1e-12 * a


def test_downsample_by_definition():
    rng = np.random.default_rng(6)
    img = rng.uniform(0, 1, (3, 11, 14))
    for n in (1, 2, 3, 4):
        out = downsample(img, n)
        assert out.shape == (3, 11 // n, 14 // n)
        for c in range(3):
            for i in range(11 // n):
                for j in range(14 // n):
                    assert abs(out[c, i, j] - img[c, i * n:(i + 1) * n, j * n:(j + 1) * n].mean()) < 1e-15
    even = img[:, :8, :12]
    assert np.allclose(downsample(even, 4).mean(axis=(1, 2)), even.mean(axis=(1, 2)), rtol=0, atol=1e-15)


def test_ratios_and_level_updates():
    r, rp = ratios([4.0, 9.0, 1.0], [2.0, 6.0, 1.0], [2.0, 3.0, 0.0])
    assert np.array_equal(r, np.float32([2.0, 3.0, np.inf]))
    assert np.array_equal(rp, np.float32([1.0, 2.0, np.inf]))
    assert TAU_F == 2.0
    # strict '<': r' = 1 raises a level, r' = 2 and inf do not; level 0 stays
    assert np.array_equal(next_levels([2, 2, 3], rp), [1, 2, 3])
    assert np.array_equal(next_levels([0, 1, 1], [0.5, 0.5, np.nan]), [0, 0, 1])


def test_sampling_follows_the_prefix_sums():
    r = np.float32([1.0, 0.0, 3.0])
    u = np.float32([0.0, 0.2, 0.25, 0.26, 0.999])
    assert np.array_equal(sample_frames(r, u), [0, 0, 2, 2, 2])  # 0.25 * 4 = 1 is not > cdf[0] = 1
    # a frame of zero weight is never drawn, whatever u
    many = sample_frames(r, np.linspace(0, 1, 1000, endpoint=False, dtype=np.float32))
    assert 1 not in many
    assert abs((many == 2).mean() - 0.75) <= 1e-3


def test_sampling_degenerate_weights():
    # no weight at all: uniform over the frames
    assert np.array_equal(sample_frames([0.0, 0.0, 0.0, 0.0], np.float32([0.0, 0.3, 0.6, 0.99])), [0, 1, 2, 3])
    # an infinite ratio is capped so the prefix sums stay finite, and dominates
    assert np.array_equal(sample_frames(np.float32([1.0, np.inf, 1.0]), np.float32([0.001, 0.5, 0.999])), [1, 1, 1])
    # NaN weighs nothing
    assert np.array_equal(sample_frames(np.float32([np.nan, 2.0]), np.float32([0.0, 0.7])), [1, 1])

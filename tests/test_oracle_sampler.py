"""Pins of the oracle's Halton(2,3) camera sampler with a per-pixel
Cranley-Patterson rotation (the sampler of the paper's wavefront renderer,
Sec. 4).

The radical inverse phi_b(n) (digits of n in base b mirrored about the radix
point, truncated to 24 bits) is pinned by values worked out by hand, by the
van der Corput stratification of its first b^k points, and by the Halton
property that the first 2^a 3^b points of (phi_2, phi_3) put exactly one point
in each cell of the 2^a x 3^b grid.  The rotation is pinned against NumPy's
Philox4x64-10 at the reserved sample index and as an exact addition modulo 1
on the 2^-24 grid.  A Halton render must estimate the same image as the
Philox render (same integrand, another point set).
"""
import numpy as np
import pytest

import oracle
from paper_2605_27323_amd import scenes
from tests.test_oracle_rng import numpy_block

ULP = 2.0 ** -24


def q24(x):
    """a value on the 2^-24 grid as its integer numerator"""
    v = int(round(x * 2 ** 24))
    assert v * ULP == x
    return v


@pytest.mark.parametrize("n,expect", [
    (0, 0.0), (1, 0.5), (2, 0.25), (3, 0.75), (6, 0.375),  # 110 -> .011
    (11, 13 / 16),  # 1011 -> .1101
    (2 ** 24 - 1, 1 - ULP), (2 ** 31, 0.0),  # bit 31 of n lands below the 24-bit grid
    (2 ** 23, ULP), (2 ** 32 - 1, 1 - ULP),
])
def test_radical_inverse_base2_hand_values(n, expect):
    assert oracle.radical_inverse(n, 2) == expect


@pytest.mark.parametrize("n,num,den", [
    (1, 1, 3), (2, 2, 3), (3, 1, 9), (5, 7, 9),  # 12_3 -> 0.21_3
    (13, 13, 27),  # 111_3 -> 0.111_3
    (26, 26, 27),  # 222_3 -> 0.222_3
])
def test_radical_inverse_base3_hand_values(n, num, den):
    # truncation: the largest multiple of 2^-24 not above num/den
    assert oracle.radical_inverse(n, 3) == (num * 2 ** 24 // den) * ULP


def test_van_der_corput_stratification():
    for k in range(1, 13):
        v = np.array([q24(oracle.radical_inverse(i, 2)) for i in range(2 ** k)])
        assert sorted(v) == [j << (24 - k) for j in range(2 ** k)]  # exactly the grid j / 2^k
    for k in range(1, 8):
        x = np.array([oracle.radical_inverse(i, 3) for i in range(3 ** k)], np.float64) * 3 ** k
        j = np.round(x)
        assert (np.abs(x - j) < 3 ** k * ULP).all() and (x <= j).all()  # truncated j / 3^k
        assert sorted(j.astype(int)) == list(range(3 ** k))


@pytest.mark.parametrize("a,b", [(1, 1), (3, 2), (4, 3), (2, 5)])
def test_halton_elementary_intervals(a, b):
    n = 2 ** a * 3 ** b
    u0 = np.array([oracle.radical_inverse(i, 2) for i in range(n)], np.float64)
    u1 = np.array([oracle.radical_inverse(i, 3) for i in range(n)], np.float64)
    # a point of phi_3 on a cell boundary is truncated just below it: lift by
    # less than the distance to any other boundary (1 / 3^digits >> 2^-20)
    cells = np.floor(u0 * 2 ** a).astype(int) * 3 ** b + np.floor((u1 + 2.0 ** -20) * 3 ** b).astype(int)
    assert sorted(cells) == list(range(n))


def test_radical_inverse_rejects_other_bases():
    with pytest.raises(Exception):
        oracle.radical_inverse(1, 5)


@pytest.mark.parametrize("seed,job", [(0, 0), (123, 3), (2 ** 63 + 5, 1)])
def test_rotation_is_the_reserved_philox_block(seed, job):
    for pix in (0, 1, 77, 2 ** 20 + 3):
        words = numpy_block((pix, 0xFFFFFFFF, 0, job), (seed, 0))
        c0 = int(words[0]) & 0xFFFFFFFF
        c1 = (int(words[0]) >> 32) & 0xFFFFFFFF
        u0, u1 = oracle.halton_jitter(seed, pix, 0, job)  # phi(0) = 0: the rotation itself
        assert q24(u0) == c0 >> 8 and q24(u1) == c1 >> 8


def test_rotation_adds_modulo_one_on_the_grid():
    rng = np.random.default_rng(4)
    for pix in rng.integers(0, 2 ** 21, 20):
        pix = int(pix)
        r0, r1 = (q24(x) for x in oracle.halton_jitter(9, pix, 0))
        for s in [1, 2, 3, 5, 36, 1000, 2 ** 24 + 7, 2 ** 32 - 2]:
            u0, u1 = (q24(x) for x in oracle.halton_jitter(9, pix, s))
            assert u0 == (r0 + q24(oracle.radical_inverse(s, 2))) % 2 ** 24
            assert u1 == (r1 + q24(oracle.radical_inverse(s, 3))) % 2 ** 24
            assert 0 <= u0 < 2 ** 24 and 0 <= u1 < 2 ** 24


def test_rotated_points_keep_the_stratification():
    # a rotation mod 1 shifts every point of a stratified set by the same
    # amount: the first 2^k (3^k) points stay one per interval, cyclically
    for pix in (3, 4000):
        r0 = oracle.halton_jitter(1, pix, 0)[0]
        u = np.sort([(oracle.halton_jitter(1, pix, i)[0] - r0) % 1.0 for i in range(64)])
        assert np.array_equal(u, np.arange(64) / 64)
        u0 = np.array([oracle.halton_jitter(1, pix, i)[0] for i in range(64)])
        assert np.array_equal(np.sort(np.floor(((u0 - r0) % 1.0) * 64)), np.arange(64))


def test_rotations_are_uniform_and_pixel_independent():
    n = 4096
    r = np.array([oracle.halton_jitter(17, p, 0) for p in range(n)])
    assert ((r >= 0) & (r < 1)).all()
    for c in range(2):
        h, _ = np.histogram(r[:, c], bins=16, range=(0, 1))
        chi2 = ((h - n / 16) ** 2 / (n / 16)).sum()
        assert chi2 < 45  # 15 degrees of freedom, p ~ 1e-4
    assert abs(np.corrcoef(r[:, 0], r[:, 1])[0, 1]) < 0.08
    assert len({tuple(x) for x in r}) == n


def test_halton_integrates_the_pixel_footprint_better_than_random():
    # u -> f(u) = u0 + u1^2 over the unit square has mean 5/6; the Halton
    # points' error falls like (log N)^2 / N, the random points' like N^-1/2
    N = 2 ** 4 * 3 ** 3
    err_h, err_r = [], []
    for pix in range(64):
        h = np.array([oracle.halton_jitter(2, pix, s) for s in range(N)], np.float64)
        err_h.append(abs((h[:, 0] + h[:, 1] ** 2).mean() - 5 / 6))
        w = [numpy_block((pix, s, 0, 0), (2, 0))[0] for s in range(N)]
        u0 = np.array([oracle.unif(int(x) & 0xFFFFFFFF) for x in w])
        u1 = np.array([oracle.unif(int(x) >> 32) for x in w])
        err_r.append(abs((u0 + u1 ** 2).mean() - 5 / 6))
    assert np.mean(err_h) < 0.2 * np.mean(err_r)
    assert max(err_h) < 3.0 / N


def test_halton_render_estimates_the_same_image():
    scene, cam = scenes.cornell()
    cam = dict(cam, width=24, height=24)
    S = oracle.Scene(scene)
    a, _ = S.render(cam, spp=64, max_depth=4, seed=1, sampler=0)
    b, _ = S.render(cam, spp=64, max_depth=4, seed=1, sampler=1)
    assert not np.array_equal(a, b)
    # image means agree to the Monte Carlo error of 24*24*64 paths
    ma, mb = a.mean(0), b.mean(0)
    assert (np.abs(ma - mb) <= 0.03 * ma).all(), (ma, mb)
    # the first vertex's jitter is the only change: D = 0 sees emitters only
    # through the pixel footprint, and an all-emissive view is exact
    fs, fc = scenes.furnace(albedo=0.5, le=1.5, n=3, width=5, height=4)
    F = oracle.Scene(fs)
    x, _ = F.render(fc, spp=3, max_depth=0, nee=False, sampler=1)
    assert np.array_equal(x, np.full_like(x, np.float32(1.5)))


def test_render_rejects_unknown_sampler():
    scene, cam = scenes.cornell()
    cam = dict(cam, width=4, height=4)
    with pytest.raises(Exception):
        oracle.Scene(scene).render(cam, spp=1, sampler=2)

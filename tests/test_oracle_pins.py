"""Pins of the CPU oracle against things other than itself (CPU only).

* brute force with exact rationals (tests/bruteforce.py) on tiny inputs,
* hand-computed cases and closed forms (Samuelson's bound and its ties),
* special cases that reduce to library routines (numpy sums, medians),
* invariants of the definitions (shift, scale, permutation, FD with one bin
  equals TD on the transpose, per-column shifts leave FD flags unchanged -- the
  paper's remark that FDSC does not affect broadband signal, Section V-A),
* statistics of noise-only input.
"""
from __future__ import annotations

import itertools
import math
import struct
from fractions import Fraction

import numpy as np
import pytest

import bruteforce as bf
import oracle

KS = [0.0, 0.5, 1.0, 1.25, 1.5, 2.0, 2.75, 3.0, 3.25, 4.0]


def rand_steps(rng, C, nsteps, masked=False):
    divs = [b for b in range(1, C + 1) if C % b == 0]
    out = []
    for _ in range(nsteps):
        dom = "td" if rng.random() < 0.5 else "fd"
        if masked and dom == "td" and rng.random() < 0.7:
            dom = "td_masked"
        k = float(rng.choice(KS)) if rng.random() < 0.7 else float(rng.uniform(0.0, 3.0))
        rep = "mean" if rng.random() < 0.5 else "median"
        b = int(rng.choice(divs)) if dom == "fd" else 0
        out.append((dom, k, rep, b))
    return out


def rand_f32(rng, shape):
    kind = rng.integers(0, 4)
    if kind == 0:
        x = rng.standard_normal(shape)
    elif kind == 1:   # wide exponent range, both signs
        x = rng.standard_normal(shape) * np.exp2(rng.integers(-60, 60, size=shape))
    elif kind == 2:   # small integers: many exact ties
        x = rng.integers(-3, 4, size=shape).astype(np.float64)
    else:             # subnormals, zeros of both signs, large values
        pool = np.array([0.0, -0.0, 1e-45, -1e-45, 3e-42, 1.5, -2.5, 1e30, -7e29, 1e-38],
                        dtype=np.float32)
        x = rng.choice(pool, size=shape)
    return x.astype(np.float32)


@pytest.mark.parametrize("seed", range(40))
def test_bruteforce_u8_random(seed):
    rng = np.random.default_rng(1000 + seed)
    C = int(rng.integers(1, 9))
    T = int(rng.integers(1, 13))
    hi = int(rng.choice([2, 8, 256]))
    x = rng.integers(0, hi, size=(C, T)).astype(np.uint8)
    steps = rand_steps(rng, C, int(rng.integers(1, 5)))
    want, wbits = bf.pipeline(x, steps)
    got, gbits = oracle.pipeline(x, steps, want_flags=True)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(gbits, wbits)


@pytest.mark.parametrize("seed", range(40))
def test_bruteforce_f32_random(seed):
    rng = np.random.default_rng(2000 + seed)
    C = int(rng.integers(1, 7))
    T = int(rng.integers(1, 11))
    x = rand_f32(rng, (C, T))
    steps = rand_steps(rng, C, int(rng.integers(1, 4)))
    want, wbits = bf.pipeline(x, steps)
    got, gbits = oracle.pipeline(x, steps, want_flags=True)
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))
    np.testing.assert_array_equal(gbits, wbits)


@pytest.mark.parametrize("seed", range(40))
def test_bruteforce_masked_u8_random(seed):
    """Masked TD steps (mixed with TD and FD steps) against the brute force."""
    rng = np.random.default_rng(7000 + seed)
    C = int(rng.integers(1, 7))
    T = int(rng.integers(1, 14))
    hi = int(rng.choice([2, 8, 256]))
    x = rng.integers(0, hi, size=(C, T)).astype(np.uint8)
    steps = rand_steps(rng, C, int(rng.integers(1, 6)), masked=True)
    want, wbits = bf.pipeline(x, steps)
    got, gbits = oracle.pipeline(x, steps, want_flags=True)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(gbits, wbits)


@pytest.mark.parametrize("seed", range(16))
def test_bruteforce_masked_f32_random(seed):
    rng = np.random.default_rng(7500 + seed)
    C = int(rng.integers(1, 6))
    T = int(rng.integers(1, 11))
    x = rand_f32(rng, (C, T))
    steps = rand_steps(rng, C, int(rng.integers(1, 5)), masked=True)
    want, wbits = bf.pipeline(x, steps)
    got, gbits = oracle.pipeline(x, steps, want_flags=True)
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))
    np.testing.assert_array_equal(gbits, wbits)


def test_first_masked_step_is_a_td_step():
    """A run's first masked step sees an empty mask: it is the plain TD step."""
    rng = np.random.default_rng(7900)
    x = rng.integers(0, 256, size=(12, 700)).astype(np.uint8)
    x[:, ::37] = 255
    for k, rep in ((2.5, "mean"), (1.0, "median"), (0.0, "mean")):
        a, fa = oracle.pipeline(x, [("td_masked", k, rep, 0)], want_flags=True)
        b, fb = oracle.pipeline(x, [("td", k, rep, 0)], want_flags=True)
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(fa, fb)


def test_masked_rows_with_every_sample_set_aside():
    """k = 0 on rows of 0s and 2s with a non-integer mean cuts every sample at
    the first masked step; later masked steps see no sample and change nothing
    (brute force, and the state after the first step)."""
    x = np.array([[0, 2, 2, 0, 2], [0, 2, 0, 2, 2], [1, 1, 1, 1, 1], [0, 2, 0, 2, 0]], np.uint8)
    steps = [("td_masked", 0.0, "mean", 0), ("td_masked", 0.0, "median", 0), ("td_masked", 1.5, "mean", 0)]
    want, wbits = bf.pipeline(x, steps)
    got, gbits = oracle.pipeline(x, steps, want_flags=True)
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(gbits, wbits)
    first, fbits = oracle.pipeline(x, steps[:1], want_flags=True)
    np.testing.assert_array_equal(got, first)
    np.testing.assert_array_equal(gbits, fbits)
    # rows 0, 1 and 3 have means 1.2 and 0.8: every sample cut and replaced by 1
    assert (got[[0, 1, 3]] == 1).all() and (gbits[[0, 1, 3]] == 1).all()
    assert (got[2] == 1).all() and (gbits[2] == 0).all()


def test_masked_run_cuts_each_sample_once():
    """Within a run of masked steps a sample is cut at most once, keeps the
    value of the step that cut it, and every sample not cut is unchanged; the
    number of set-aside samples never falls."""
    rng = np.random.default_rng(7901)
    x = np.clip(rng.normal(100, 12, size=(16, 900)), 0, 255).astype(np.uint8)
    x[rng.random(x.shape) < 0.03] = 250
    steps = [("td_masked", 2.0, "mean", 0)] * 5
    out, fl = oracle.pipeline(x, steps, want_flags=True)
    bits = np.unpackbits(fl[..., None], axis=-1).sum(axis=-1)
    assert bits.max() == 1 and bits.sum() > 0
    untouched = fl == 0
    np.testing.assert_array_equal(out[untouched], x[untouched])
    counts = [int(((fl >> j) & 1).sum()) for j in range(5)]
    assert counts[0] > 0 and all(c >= 0 for c in counts)
    for c in range(x.shape[0]):
        for j in range(5):
            cut = ((fl[c] >> j) & 1).astype(bool)
            if cut.any():   # one replacement value per row and step
                assert len(set(out[c][cut].tolist())) == 1


def test_exhaustive_small_rows():
    """Every row of 4 values in 0..4 under TD at several k, mean and median."""
    rows = np.array(list(itertools.product(range(5), repeat=4)), dtype=np.uint8)
    for k in (0.0, 0.5, 1.0, 1.2, 1.5):
        for rep in ("mean", "median"):
            want, wf = bf.td_step(rows, k, rep)
            got, gf = oracle.td_step(rows, k, rep)
            np.testing.assert_array_equal(got, want)
            np.testing.assert_array_equal(gf.astype(bool), wf)


def test_hand_td_ten_samples():
    """Row [0 x9, 10]: mu = 1, sigma = 3 (population).  At k = 3.25 the last
    sample is inside (9 < 9.75); at 2.75 it is out (9 > 8.25) and becomes
    round(1) = 1; a second 2.75 step sees mu = 0.1, sigma = 0.3 and replaces
    the 1 with round(0.1) = 0; a third step sees a constant row."""
    x = np.array([[0] * 9 + [10]], dtype=np.uint8)
    out, fl = oracle.td_step(x, 3.25)
    assert (out == x).all() and not fl.any()
    out, fl = oracle.pipeline(x, [("td", 2.75, "mean", 0)] * 3, want_flags=True)
    assert (out == 0).all()
    assert fl[0, 9] == 0b011 and not fl[0, :9].any()


def test_hand_fd_eight_channels():
    """Column [5,5,5,5, 5,5,5,25], bins of 4: bin means 5 and 10, mean-corrected
    values 0,0,0,0,-5,-5,-5,15 with mean 0 and variance 37.5.  Channel 7 has
    15^2 = 225 > 2.25^2 * 37.5 = 189.84 but not > 2.75^2 * 37.5 = 283.59; it is
    replaced by its bin mean 10 (the original value, not the corrected one)."""
    col = np.array([5, 5, 5, 5, 5, 5, 5, 25], dtype=np.uint8).reshape(8, 1)
    out, fl = oracle.fd_step(col, 2.25, 4)
    assert out[:, 0].tolist() == [5, 5, 5, 5, 5, 5, 5, 10]
    assert fl[:, 0].tolist() == [0] * 7 + [1]
    out, fl = oracle.fd_step(col, 2.75, 4)
    assert (out == col).all() and not fl.any()
    out, fl = oracle.fd_step(col + 17, 2.25, 4)     # broadband offset: same flags
    assert fl[:, 0].tolist() == [0] * 7 + [1] and out[7, 0] == 27


@pytest.mark.parametrize("k", [2.75, 3.0, 3.25, 3.5, 4.0])
def test_samuelson_single_outlier(k):
    """One value v among n-1 zeros sits exactly sqrt(n-1) population standard
    deviations from the mean, so it is flagged iff n - 1 > k^2 (strict).  The
    ties n = 10 at k = 3 and n = 17 at k = 4 are not flagged; a sample
    standard deviation (n - 1 denominator) would flag them."""
    for n in range(2, 30):
        for v in (1, 7, 255):
            x = np.zeros((1, n), dtype=np.uint8)
            x[0, n // 2] = v
            _, fl = oracle.td_step(x, k)
            assert bool(fl[0, n // 2]) == (n - 1 > k * k), (n, v)
            assert fl.sum() == fl[0, n // 2]


def test_samuelson_bound_no_flags():
    """|x - mu| <= sigma * sqrt(n - 1): with k^2 >= n - 1 nothing can flag."""
    rng = np.random.default_rng(7)
    for n in (2, 5, 9, 10, 17):
        x = rng.integers(0, 256, size=(200, n)).astype(np.uint8)
        _, fl = oracle.td_step(x, math.sqrt(n - 1) + 1e-12)
        assert not fl.any()


def test_constant_rows_never_flag():
    x = np.full((3, 50), 77, dtype=np.uint8)
    for k in (0.0, 1.0, 3.25):
        out, fl = oracle.td_step(x, k)
        assert not fl.any() and (out == x).all()
        out, fl = oracle.fd_step(x.T.copy(), k, 0)
        assert not fl.any()


def test_k_zero_flags_everything_off_mean():
    """k = 0 flags exactly the samples that differ from the mean; with median
    replacement they take the value numpy's partition gives."""
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, size=(20, 31)).astype(np.uint8)
    out, fl = oracle.td_step(x, 0.0, "median")
    med = np.partition(x, 15, axis=1)[:, 15]
    mean_is = x.sum(axis=1) % 31 == 0
    for c in range(20):
        off = x[c] * 31 != x[c].sum() if mean_is[c] else np.ones(31, bool)
        assert (fl[c].astype(bool) == off).all()
        assert (out[c][off] == med[c]).all()


def test_mean_matches_library_sums():
    """uint8 mean replacement = round-half-even of numpy's exact int64 sum / n;
    float32 mean = nearest float32 to the exact rational sum / n."""
    rng = np.random.default_rng(11)
    for n in (1, 2, 3, 4, 7, 100, 12500):
        x = rng.integers(0, 256, size=n).astype(np.uint8)
        s = int(np.sum(x, dtype=np.int64))
        assert oracle.mean_u8(x) == round(Fraction(s, n))
    for n in (2, 4):          # exact .5 ties go to even
        assert oracle.mean_u8(np.array([0, 1] * (n // 2), np.uint8)) == 0
        assert oracle.mean_u8(np.array([1, 2] * (n // 2), np.uint8)) == 2
    for n in (1, 3, 10, 1000):
        x = (rng.standard_normal(n) * 1000).astype(np.float32)
        exact = sum((Fraction(float(v)) for v in x), Fraction(0)) / n
        # math.fsum gives the exact sum rounded once; for these sizes the
        # rational mean's nearest float32 must agree with the brute force.
        assert oracle.mean_f32(x) == bf.nearest_f32(exact)
        assert abs(float(oracle.mean_f32(x)) - math.fsum(float(v) for v in x) / n) <= \
            abs(float(np.spacing(np.float32(exact))))


def test_f32_mean_subnormal_and_ties():
    tiny = np.float32(1e-45)                       # 2^-149, the smallest subnormal
    assert oracle.mean_f32(np.array([tiny, 0.0], np.float32)) == 0.0      # tie -> even (0)
    three = np.float32(3 * 1e-45)
    assert oracle.mean_f32(np.array([three, 0.0], np.float32)) == np.float32(2 * 1e-45)
    big = np.float32(2.0 ** 24)
    one = np.float32(1.0)
    # (2^24 + 1)/2 is a tie between 2^23 and 2^23 + 1: ties to the even mantissa
    assert oracle.mean_f32(np.array([big + 0, one], np.float32) * 1) == np.float32((2 ** 24 + 1) / 2)


def test_fd_one_bin_equals_td_transposed():
    """With one bin spanning every channel the mean-corrected samples are the
    column minus its mean, so FD is TD applied to the transposed array."""
    rng = np.random.default_rng(5)
    for dt in (np.uint8, np.float32):
        x = (rng.integers(0, 256, size=(24, 40)) if dt == np.uint8 else
             rng.standard_normal((24, 40)) * 3).astype(dt)
        for k in (1.0, 2.0, 2.75):
            for rep in ("mean", "median"):
                a, fa = oracle.fd_step(x, k, 0, rep)
                b, fb = oracle.td_step(np.ascontiguousarray(x.T), k, rep)
                np.testing.assert_array_equal(a.view(np.uint8), np.ascontiguousarray(b.T).view(np.uint8))
                np.testing.assert_array_equal(fa, fb.T)


def test_td_shift_and_scale_invariance():
    rng = np.random.default_rng(9)
    x = rng.integers(0, 200, size=(16, 300)).astype(np.uint8)
    x[:, ::37] = 199
    steps = [("td", 2.0, "mean", 0), ("td", 1.5, "median", 0)]
    a, fa = oracle.pipeline(x, steps, True)
    # even shifts: round-half-even commutes with adding an even integer
    shift = (2 * rng.integers(0, 28, size=(16, 1))).astype(np.uint8)
    b, fb = oracle.pipeline(x + shift, steps, True)
    np.testing.assert_array_equal(fa, fb)
    np.testing.assert_array_equal(b, a + shift)
    xf = rng.standard_normal((8, 500)).astype(np.float32)
    a, fa = oracle.pipeline(xf, steps, True)
    b, fb = oracle.pipeline(xf * np.float32(2.0 ** 7), steps, True)
    np.testing.assert_array_equal(fa, fb)
    np.testing.assert_array_equal(b, a * np.float32(2.0 ** 7))


def test_fd_per_column_shift_leaves_flags():
    """Adding the same value to every channel of a time sample (a broadband
    signal) changes neither the FD flags nor which channels are replaced."""
    rng = np.random.default_rng(13)
    x = rng.integers(0, 150, size=(64, 200)).astype(np.uint8)
    x[5, :] = 149
    x[40:42, 50:60] = 0
    steps = [("fd", 2.0, "mean", 16), ("fd", 1.75, "median", 8)]
    a, fa = oracle.pipeline(x, steps, True)
    shift = (2 * rng.integers(0, 50, size=(1, 200))).astype(np.uint8)   # even: see TD test
    b, fb = oracle.pipeline(x + shift, steps, True)
    np.testing.assert_array_equal(fa, fb)
    np.testing.assert_array_equal(b, a + shift)


def test_permutation_equivariance():
    rng = np.random.default_rng(17)
    x = rng.integers(0, 256, size=(6, 200)).astype(np.uint8)
    perm = rng.permutation(200)
    for rep in ("mean", "median"):
        a, fa = oracle.td_step(x, 1.5, rep)
        b, fb = oracle.td_step(x[:, perm], 1.5, rep)
        np.testing.assert_array_equal(a[:, perm], b)
        np.testing.assert_array_equal(fa[:, perm], fb)
    cperm = np.concatenate([rng.permutation(8) + 8 * b for b in range(4)])   # within bins
    a, fa = oracle.fd_step(np.ascontiguousarray(x[:, :32].T), 1.5, 8)
    b, fb = oracle.fd_step(np.ascontiguousarray(x[:, :32].T[cperm]), 1.5, 8)
    np.testing.assert_array_equal(a[cperm], b)
    np.testing.assert_array_equal(fa[cperm], fb)


def test_iteration_reaches_fixed_point():
    """With mean replacement the spread D = n*S2 - S1^2 (a non-negative integer
    for uint8) drops whenever a sample is replaced, so repeated TD steps stop
    changing the data; at that point one more step is the identity."""
    rng = np.random.default_rng(19)
    x = rng.integers(0, 256, size=(10, 64)).astype(np.uint8)
    cur = x
    for it in range(400):
        nxt, fl = oracle.td_step(cur, 1.0)
        if not fl.any():
            break
        d_prev = 64 * (cur.astype(np.int64) ** 2).sum(1) - cur.astype(np.int64).sum(1) ** 2
        d_next = 64 * (nxt.astype(np.int64) ** 2).sum(1) - nxt.astype(np.int64).sum(1) ** 2
        rows = fl.any(1)
        assert (d_next[rows] < d_prev[rows]).all()
        cur = nxt
    else:
        pytest.fail("no fixed point")
    again, fl = oracle.td_step(cur, 1.0)
    assert not fl.any() and (again == cur).all()


def test_noise_flag_rate_matches_gaussian_tail():
    """On N(0,1) float32 noise one TD step at k flags a fraction close to
    2*Q(k) = erfc(k/sqrt(2)) (statistical, 5-sigma binomial bound)."""
    rng = np.random.default_rng(23)
    x = rng.standard_normal((4, 50000)).astype(np.float32)
    for k in (2.75, 3.25):
        _, fl = oracle.td_step(x, k)
        p = math.erfc(k / math.sqrt(2.0))
        n = x.size
        assert abs(fl.sum() - p * n) < 5 * math.sqrt(n * p * (1 - p)) + 5


def test_rejects_bad_arguments():
    x = np.zeros((4, 4), np.uint8)
    for st in ([("td", -1.0, "mean", 0)], [("td", float("nan"), "mean", 0)],
               [("fd", 1.0, "mean", 3)], [("td", float("inf"), "mean", 0)]):
        with pytest.raises(ValueError):
            oracle.pipeline(x, st)
    with pytest.raises(ValueError):
        oracle.pipeline(x, [("td", 1.0, "mean", 0)] * 9, want_flags=True)


def test_padding_columns_untouched():
    rng = np.random.default_rng(29)
    x = rng.integers(0, 256, size=(8, 40)).astype(np.uint8)
    out, fl = oracle.pipeline(x, [("td", 1.0, "mean", 0), ("fd", 1.0, "mean", 4)], True, nsamp=33)
    np.testing.assert_array_equal(out[:, 33:], x[:, 33:])
    assert not fl[:, 33:].any()
    ref, rfl = oracle.pipeline(np.ascontiguousarray(x[:, :33]), [("td", 1.0, "mean", 0), ("fd", 1.0, "mean", 4)], True)
    np.testing.assert_array_equal(out[:, :33], ref)
    np.testing.assert_array_equal(fl[:, :33], rfl)


def test_k_is_taken_exactly():
    """k = 3 exactly ties at n = 10; the next double above 3 still ties in
    real arithmetic only if rounded, so it must not flag, and the double just
    below 3 must flag."""
    x = np.zeros((1, 10), np.uint8)
    x[0, 0] = 9
    assert not oracle.td_step(x, 3.0)[1].any()
    assert not oracle.td_step(x, np.nextafter(3.0, 4.0))[1].any()
    assert oracle.td_step(x, np.nextafter(3.0, 0.0))[1].any()

"""Brute-force sigma cuts on tiny inputs with exact rationals (fractions).

Written straight from the definitions of Section IV of the paper, in a
different form from the oracle: the mean and the variance are computed as
mu = sum(x)/n and var = sum((x - mu)^2)/n (two passes), an outlier satisfies
(x - mu)^2 > k^2 * var, and the FD step runs the same test on the
mean-corrected samples y_c = x_c - (bin mean).  Used only to pin the oracle.
"""
from __future__ import annotations

import struct
from fractions import Fraction

import numpy as np


def f32_exact(v) -> Fraction:
    return Fraction(float(np.float32(v)))


def total_order_key(v):
    u = struct.unpack("<I", struct.pack("<f", float(v)))[0]
    return (~u & 0xFFFFFFFF) if u & 0x80000000 else (u | 0x80000000)


def nearest_f32(q: Fraction) -> np.float32:
    """float32 nearest to the rational q, ties to an even mantissa."""
    d = float(q)  # correctly rounded to double by Python
    cand = {np.float32(d)}
    for c in list(cand):
        cand.add(np.nextafter(c, np.float32(np.inf)))
        cand.add(np.nextafter(c, np.float32(-np.inf)))
    cand = [c for c in cand if np.isfinite(c)]
    best = min(abs(Fraction(float(c)) - q) for c in cand)
    ties = [c for c in cand if abs(Fraction(float(c)) - q) == best]
    if len(ties) > 1:
        ties = [c for c in ties if (struct.unpack("<I", struct.pack("<f", float(c)))[0] & 1) == 0]
    return np.float32(ties[0])


def round_dtype(q: Fraction, dtype):
    if dtype == np.uint8:
        return np.uint8(round(q))      # Python rounds Fractions half to even
    return nearest_f32(q)


def lower_median(vals, dtype):
    if dtype == np.uint8:
        s = sorted(int(v) for v in vals)
    else:
        s = sorted((np.float32(v) for v in vals), key=total_order_key)
    return s[(len(s) - 1) // 2]


def outliers(vals, k):
    """Indices i with |v_i - mean| > k * std (population), exactly."""
    n = len(vals)
    mu = sum(vals, Fraction(0)) / n
    var = sum(((v - mu) ** 2 for v in vals), Fraction(0)) / n
    kk = Fraction(float(k)) ** 2
    return [(v - mu) ** 2 > kk * var for v in vals], mu


def td_step(x: np.ndarray, k, replace="mean"):
    out = x.copy()
    flags = np.zeros(x.shape, dtype=bool)
    for c in range(x.shape[0]):
        row = x[c]
        vals = [Fraction(int(v)) if x.dtype == np.uint8 else f32_exact(v) for v in row]
        fl, mu = outliers(vals, k)
        r = round_dtype(mu, x.dtype) if replace == "mean" else lower_median(row, x.dtype)
        for t, f in enumerate(fl):
            if f:
                out[c, t] = r
                flags[c, t] = True
    return out, flags


def td_step_masked(x: np.ndarray, k, replace, mask):
    """Masked TD step: per row, only the samples with mask False take part;
    the cut ones are replaced and join the mask (mask is updated in place)."""
    out = x.copy()
    flags = np.zeros(x.shape, dtype=bool)
    for c in range(x.shape[0]):
        idx = [t for t in range(x.shape[1]) if not mask[c, t]]
        if not idx:
            continue
        row = x[c, idx]
        vals = [Fraction(int(v)) if x.dtype == np.uint8 else f32_exact(v) for v in row]
        fl, mu = outliers(vals, k)
        r = round_dtype(mu, x.dtype) if replace == "mean" else lower_median(row, x.dtype)
        for t, f in zip(idx, fl):
            if f:
                out[c, t] = r
                flags[c, t] = True
                mask[c, t] = True
    return out, flags


def fd_step(x: np.ndarray, k, bin_size=32, replace="mean"):
    C, T = x.shape
    B = C if bin_size == 0 else bin_size
    out = x.copy()
    flags = np.zeros(x.shape, dtype=bool)
    for t in range(T):
        col = x[:, t]
        vals = [Fraction(int(v)) if x.dtype == np.uint8 else f32_exact(v) for v in col]
        means = [sum(vals[b * B:(b + 1) * B], Fraction(0)) / B for b in range(C // B)]
        y = [vals[c] - means[c // B] for c in range(C)]
        fl, _ = outliers(y, k)
        for c, f in enumerate(fl):
            if f:
                b = c // B
                out[c, t] = (round_dtype(means[b], x.dtype) if replace == "mean"
                             else lower_median(col[b * B:(b + 1) * B], x.dtype))
                flags[c, t] = True
    return out, flags


def pipeline(x: np.ndarray, steps):
    """steps: iterable of (domain, k, replace, bin_size).  Returns (out, flagbits)."""
    cur = x.copy()
    bits = np.zeros(x.shape, dtype=np.uint8)
    mask = None
    for j, (dom, k, rep, b) in enumerate(steps):
        if dom == "td_masked":
            if j == 0 or steps[j - 1][0] != "td_masked":
                mask = np.zeros(x.shape, dtype=bool)   # a new run of masked steps
            cur, fl = td_step_masked(cur, k, rep, mask)
        elif dom == "td":
            cur, fl = td_step(cur, k, rep)
        else:
            cur, fl = fd_step(cur, k, b, rep)
        bits |= (fl.astype(np.uint8) << j)
    return cur, bits

"""Helpers of the GPU parity tests (inputs on the device, oracle bounds)."""
import numpy as np
import torch

from oracle import fd

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def to_dev(entries, dtype):
    np_dt = np.float32 if dtype == torch.float32 else np.float64
    host = [np.ascontiguousarray(E, dtype=np_dt) for E in entries]
    return host, [torch.from_numpy(E).to("cuda") for E in host]


def oracle_inputs(host):
    """Reading for FP32 inputs: the oracle sees the same rounded entries, widened exactly."""
    return [E.astype(np.float64) for E in host]


def abs_bound(entries64, cut, xs=None):
    """T_x = 2^-K sum_l prod_c |E_c| : scale of every rounding error at output x."""
    return fd.reconstruct([np.abs(E) for E in entries64], cut, xs)


def elementwise_ok(p, ref, T, unit, terms):
    """|p - ref| <= 4 (terms + 2) u T_x, the bound of any order of the term sum
    with one rounding per multiply and per add."""
    tol = 4.0 * (terms + 2) * unit * T
    err = np.abs(np.asarray(p, dtype=np.float64) - ref)
    bad = np.nonzero(err > tol)[0]
    return bad.size == 0, (bad[:5], err[bad[:5]] if bad.size else None, tol[bad[:5]] if bad.size else None)


def sum_terms(prec, t):
    """Roundings an output of t terms goes through: the BF16X6 form adds six
    partial products per term, and its three-part split (exact) drops products
    below about 2^-24 |a b| = u |a b| per term (one more u-multiple of T_x).
    The BF16X3 form adds three, and its two-part split (remainder at most
    2^-17 |a|, first part's remainder at most 2^-8 |a|) drops up to
    (2^-16 + 2 * 2^-17) |a b| = 2^-15 |a b| = 512 u |a b| per term: 128 more
    u-multiples of T_x under the factor 4 of elementwise_ok (the bounds are
    checked on the host in test_split_bound)."""
    if prec == "bf16x6":
        return 6 * t + 1
    if prec == "bf16x3":
        return 3 * t + 128
    return t


# relative L1 bar of each precision: the flat 1e-6 target for FP32 and
# BF16X6; for BF16X3 its dropped part (2^-15 = 3.05e-5 of T_x at most), which
# the tests scale by kappa = sum T_x / sum |p_x|
REL_L1 = {"fp32": 1e-6, "bf16x6": 1e-6, "bf16x3": 3.1e-5}

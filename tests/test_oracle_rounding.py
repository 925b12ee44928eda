"""Pins of the oracle's value rounding (binary32 and bfloat16, nearest-even)
against hand-derived bit patterns and against independent library
conversions (numpy float32, torch bfloat16 from float32)."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_bf16_golden_cases():
    d = json.load(open(os.path.join(HERE, "golden", "bf16_rounding.json")))
    xs = np.array([float.fromhex(c["x"]) for c in d["cases"]])
    want = np.array([int(c["bits"], 16) for c in d["cases"]], np.uint16)
    got = oracle.round_bf16(xs)
    bad = [(c["x"], hex(g), c["bits"]) for c, g in zip(d["cases"], got) if g != int(c["bits"], 16)]
    assert not bad


def _interesting_doubles(n, seed):
    u = synth.uniform(n, seed, 1, -1, 1)
    e = (synth.u64(seed, 2, n) % np.uint64(300)).astype(np.int64) - 150
    return np.ldexp(u, e)


def test_bf16_matches_torch_on_binary32_inputs():
    """For values already exactly binary32, rounding to bfloat16 must agree
    with torch's float32 -> bfloat16 conversion (nearest-even)."""
    torch = pytest.importorskip("torch")
    with np.errstate(over="ignore"):  # values past the binary32 range become inf and are dropped
        f = _interesting_doubles(200_000, 3).astype(np.float32)
    f = f[np.isfinite(f)]
    want = torch.from_numpy(f).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    got = oracle.round_bf16(f.astype(np.float64))
    assert np.array_equal(got, want)


def test_bf16_is_nearest_on_doubles():
    """For arbitrary doubles the result is a neighbour of x on the bfloat16
    grid and no other bfloat16 value is closer (ties: even significand)."""
    x = _interesting_doubles(50_000, 4)
    x = x[np.abs(x) < 3.3e38]
    b = oracle.round_bf16(x).astype(np.int64)
    def val(bits):
        return oracle.bf16_to_f64(np.asarray(bits % 65536, np.uint16))
    r = val(b)
    # the two neighbours in bit space (same sign): b-1 and b+1 magnitudes
    up, dn = val(b + 1), val(b - 1)
    d0 = np.abs(r - x)
    ok_up = np.isnan(up) | np.isinf(up) | (np.abs(up - x) >= d0)
    ok_dn = (np.abs(dn - x) >= d0) | ((b % 32768) == 0)
    assert np.all(ok_up & ok_dn)
    tie = (np.abs(up - x) == d0) | (np.abs(dn - x) == d0)
    assert np.all((b[tie] & 1) == 0)


def test_f32_matches_numpy():
    x = _interesting_doubles(200_000, 5)
    with np.errstate(over="ignore"):
        want = x.astype(np.float32)
    assert np.array_equal(oracle.round_f32(x).view(np.uint32), want.view(np.uint32))


def test_bf16_roundtrip_exact():
    bits = np.arange(0, 65536, dtype=np.uint32).astype(np.uint16)
    v = oracle.bf16_to_f64(bits)
    finite = np.isfinite(v)
    again = oracle.round_bf16(v[finite])
    # +0 and -0 both map to themselves; every finite pattern is a fixed point
    assert np.array_equal(again, bits[finite])


def test_f32_golden_cases():
    """Binary32 rounding against encodings derived by hand (ties to even,
    the overflow threshold, the subnormal range, signed zeros)."""
    d = json.load(open(os.path.join(HERE, "golden", "f32_rounding.json")))
    xs = np.array([float(c["x"]) if "inf" in c["x"] else float.fromhex(c["x"]) for c in d["cases"]])
    got = oracle.round_f32(xs).view(np.uint32)
    bad = [(c["x"], hex(int(g)), c["bits"]) for c, g in zip(d["cases"], got) if int(g) != int(c["bits"], 16)]
    assert not bad


def test_f32_nan_stays_nan():
    got = oracle.round_f32(np.array([np.nan, -np.nan])).view(np.uint32)
    assert np.all((got & 0x7F800000) == 0x7F800000) and np.all((got & 0x007FFFFF) != 0)

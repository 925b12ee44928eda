"""The code-balance model (Sect. 4) against the paper's own numbers and
against algebraic round trips."""
import json
import os

import pytest

from paper_1307_6209_amd import model

HERE = os.path.dirname(os.path.abspath(__file__))


def test_best_attainable_matches_paper():
    d = json.load(open(os.path.join(HERE, "golden", "paper_model.json")))
    for dev in d["devices"]:
        b = max(dev["copy_gbs"], dev["read_gbs"])
        assert round(model.best_attainable(b, 1.0), 1) == dev["pbar_gfs"], dev["name"]


def test_crs_balance_is_beta_one():
    assert model.crs_balance(0.3, 7.0) == model.sell_balance(0.3, 1.0, 7.0) == 6 + 4 * 0.3 + 8 / 7.0


@pytest.mark.parametrize("alpha,beta,nnzr", [(1 / 7.08, 0.54, 7.08), (1.0, 1.0, 3.81), (0.5, 0.92, 98.16)])
def test_alpha_round_trip(alpha, beta, nnzr):
    nnz = 1_000_000
    V = model.sell_balance(alpha, beta, nnzr) * 2 * nnz
    assert abs(model.alpha_from_volume(V, nnz, beta, nnzr) - alpha) < 1e-12


def test_general_balance_reduces_to_paper():
    s = model.Sizes(sv=8, si=4, sx=8, sy=16, sp=0, meta=0)
    for alpha, beta, nnzr in [(0.1, 0.7, 5.0), (1.0, 1.0, 27.0)]:
        assert abs(model.general_balance(alpha, beta, nnzr, C=32, k=1, s=s) - model.sell_balance(alpha, beta, nnzr)) < 1e-12


@pytest.mark.parametrize("k", [1, 4, 32])
def test_general_alpha_round_trip(k):
    s = model.sizes_for("f64", "f64", True)
    nnz, beta, nnzr, C, alpha = 5_000_000, 0.8, 4.2, 32, 2.5
    V = model.general_balance(alpha, beta, nnzr, C, k, s) * 2 * nnz * k
    assert abs(model.general_alpha_from_volume(V, nnz, beta, nnzr, C, k, s) - alpha) < 1e-9


def test_algorithmic_bytes_27pt():
    """27-point stencil 160^3, SELL-32-1, FP64: 12 B per stored slot, x and
    y once, 12 B of chunk metadata per chunk."""
    n, padded = 160 ** 3, 109_672_320
    nb = model.algorithmic_bytes(n, n, padded, n // 32, 1, model.sizes_for("f64", "f64", False))
    assert nb == 12 * padded + 8 * n + 8 * n + 12 * (n // 32)


def test_window_sizes():
    """With the x window the streamed index is 2 bytes and each chunk carries
    its share of the window tables (8 bytes per group of 4 or 8 chunks, 12
    per segment)."""
    s = model.sizes_for("f64", "f64", False, xwindow=True, segments_per_chunk=2.5)
    assert (s.sv, s.si, s.sx, s.sy, s.sp) == (8, 2, 8, 8, 0)
    assert s.meta == 12 + 2 + 30
    b = model.algorithmic_bytes(100, 100, 1000, 10, 1, s)
    assert b == 10 * 1000 + 8 * 100 + 8 * 100 + 44 * 10
    s8 = model.sizes_for("f64", "f64", False, xwindow=True, segments_per_chunk=2.5, group_chunks=8)
    assert s8.meta == 12 + 1 + 30

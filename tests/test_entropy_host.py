"""The host rANS coder of the compression back end (C++ in libqg, no GPU): lossless round trips and a coded
size within 1% of the empirical entropy; pins of the storage oracle."""
import numpy as np
import pytest

from oracle import entropy as OE


@pytest.fixture(scope="module")
def qg():
    from paper_2412_04469_amd import qg
    return qg


def _hist(sym, L):
    h, ovf = OE.histograms(sym.reshape(-1, L).astype(np.int64))
    assert ovf == 0
    return np.ascontiguousarray(h.astype(np.uint32))


@pytest.mark.parametrize("case", ["laplace", "single", "uniform256", "tiny", "skewed"])
def test_round_trip(qg, case):
    rng = np.random.default_rng(len(case))
    L = 8
    if case == "laplace":
        sym = np.clip(np.rint(rng.laplace(0, 1.5, 80_000)), -128, 127)
    elif case == "single":
        sym = np.full(4_000, 3)
    elif case == "uniform256":
        sym = rng.integers(-128, 128, 40_000)
    elif case == "tiny":
        sym = rng.integers(-2, 3, 8)
    else:
        sym = np.where(rng.random(64_000) < 0.999, 0, rng.integers(-128, 128, 64_000))
    sym = np.ascontiguousarray(sym.astype(np.int8))
    hist = _hist(sym, L)
    data = qg.qg_rans_encode(L, sym, hist)
    back = qg.qg_rans_decode(sym.size, L, data, hist)
    assert np.array_equal(back, sym)


def test_size_within_one_percent_of_entropy(qg):
    rng = np.random.default_rng(7)
    L = 8
    scales = np.array([0.3, 0.7, 1.0, 1.5, 2.0, 3.0, 5.0, 0.1])
    sym = np.clip(np.rint(rng.laplace(0, 1.0, (250_000, L)) * scales), -128, 127).astype(np.int8).ravel()
    hist = _hist(sym, L)
    data = qg.qg_rans_encode(L, sym, hist)
    bits = OE.empirical_entropy_bits(hist.astype(np.int64))
    assert data.size * 8 <= bits * 1.01 + 64, (data.size * 8, bits)
    assert data.size * 8 >= bits - 1


def test_corrupt_stream_is_rejected(qg):
    rng = np.random.default_rng(3)
    sym = np.ascontiguousarray(np.clip(np.rint(rng.laplace(0, 2.0, 8_000)), -128, 127).astype(np.int8))
    hist = _hist(sym, 8)
    data = qg.qg_rans_encode(8, sym, hist)
    with pytest.raises(Exception):
        qg.qg_rans_decode(sym.size, 8, data[:-3].copy(), hist)


def test_oracle_entropy_and_symbols_closed_forms():
    h = np.zeros((2, 256), np.int64)
    h[0, 128] = 8           # one symbol: 0 bits
    h[1, [120, 130]] = 4    # two equiprobable symbols: 1 bit each
    assert OE.empirical_entropy_bits(h) == 8.0
    lat = np.array([[0.5, 1.5, -2.5, 2.49, -0.51], [127.4, -128.4, 127.6, 0.0, -0.0]])
    sym = OE.latent_symbols(lat)
    assert sym[:, 0].tolist() == [0, 2, -2, 2, -1]  # round half to even
    hh, ovf = OE.histograms(sym)
    assert ovf == 1 and hh.sum() == 9
    assert OE.coo_nonzero(np.array([0.0, 0.3, 0.0, 1.0])).tolist() == [1, 3]

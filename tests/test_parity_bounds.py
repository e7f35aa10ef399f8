"""CPU checks of the error bounds the GPU parity tests use (tests/parity.py), against
emulations of the arithmetic they bound: the bound must hold for the emulated kernel
arithmetic and must fail when a term of that arithmetic is dropped."""
import numpy as np

from tests import parity


def _split16(x, scale):
    """hi and lo binary16 parts of the FP32 values x scaled by an exact power of two"""
    xs = (np.asarray(x, np.float32) * np.float32(scale)).astype(np.float32)
    hi = xs.astype(np.float16)
    lo = (xs - hi.astype(np.float32)).astype(np.float16)
    return hi.astype(np.float64), lo.astype(np.float64)


def _split_cepstrum(L, D, drop=None):
    """Lh Dh + Lh Dl + Ll Dh with exact products summed in FP32 (in input order), / 2^19"""
    Lh, Ll = _split16(L, 2.0 ** 9)
    Dh, Dl = _split16(D, 2.0 ** 10)
    terms = [("hh", Lh, Dh), ("hl", Lh, Dl), ("lh", Ll, Dh)]
    T, M = L.shape
    acc = np.zeros((T, D.shape[0]), np.float32)
    for i in range(M):
        for name, a, b in terms:
            if name == drop:
                continue
            acc = (acc + (a[:, i:i + 1] * b[None, :, i]).astype(np.float32)).astype(np.float32)
    return acc.astype(np.float64) / 2.0 ** 19


def test_split_cepstrum_bound_holds_and_is_tight(orc):
    rng = np.random.default_rng(7)
    T, M, K = 48, 128, 40
    # log-Mel values over the range the log epilogue produces (eps = 1e-10 floor to loud bins),
    # with a few tiny ones whose low parts fall below binary16's normal range
    L = rng.uniform(-23.0, 20.0, size=(T, M)).astype(np.float32)
    L[:, ::17] = rng.uniform(-1e-3, 1e-3, size=L[:, ::17].shape).astype(np.float32)
    L = L.astype(np.float64)
    D = orc.dct2_ortho(K, M).astype(np.float32).astype(np.float64)
    bL = np.zeros_like(L)
    parity.check_cepstrum(_split_cepstrum(L, D), L, bL, D, label="split", split=True)
    for drop in ("hl", "lh"):
        try:
            parity.check_cepstrum(_split_cepstrum(L, D, drop=drop), L, bL, D, label=drop, split=True)
        except AssertionError:
            continue
        raise AssertionError(f"the split bound does not catch a dropped {drop} term")

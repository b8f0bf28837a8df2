"""CPU check of the identity the FX16 encode relies on: clamping a binary32
value v to [-32767, 32767] (a NaN to -32767) and adding 1.5 * 2^23 in binary32
leaves in the low 16 bits of the sum's bit pattern the int16 code
round-half-even(v), saturated at +-32767 -- the code of rounding, clamping
and converting.  numpy's binary32 addition rounds to nearest even, as the
GPU's does."""
import numpy as np


def _reference(v):
    r = np.rint(v.astype(np.float64))          # half to even
    r = np.where(np.isnan(v), -32767.0, np.clip(r, -32767.0, 32767.0))
    return r.astype(np.int64).astype(np.int16)


def _trick(v):
    c = np.where(np.isnan(v), np.float32(-32767.0),
                 np.clip(v, np.float32(-32767.0), np.float32(32767.0))).astype(np.float32)
    s = (c + np.float32(12582912.0)).astype(np.float32)
    return (s.view(np.uint32) & np.uint32(0xFFFF)).astype(np.uint16).view(np.int16)


def test_fx16_encode_identity():
    rng = np.random.default_rng(0)
    k = np.arange(-33000, 33001, dtype=np.float64)
    v = np.concatenate([
        k, k + 0.5, k - 0.5, k + 0.25, k + 0.75,                    # ties and quarters
        np.nextafter(k + 0.5, np.inf), np.nextafter(k + 0.5, -np.inf),
        rng.uniform(-40000.0, 40000.0, 200000),
        rng.normal(0.0, 50.0, 200000),                               # the usual range of codes
        [0.0, -0.0, 1e-30, -1e-30, 3e38, -3e38, np.inf, -np.inf, np.nan],
    ]).astype(np.float32)
    assert np.array_equal(_trick(v), _reference(v))

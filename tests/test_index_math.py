"""The integer divisions the kernels replace by multiplications, checked on the host over
the ranges the kernels rely on (the formulas are those stated beside each helper in
paper_1001_3764_amd/csrc/md_internal.h):

- stencil offsets: code -> (code % W, code / W % W, code / W^2) for W = 2R + 1 <= 15, from
  FP32 products (code + 1/2) * rcp(W) and (code + 1/2) * rcp(W^2); the hardware reciprocal
  is within 1 ulp, so every reciprocal within 1 ulp of the true one is tried;
- cell coordinates: lc -> (lc % M0, lc / M0 % M1, lc / (M0 M1)) from FP64 products with the
  host's 1/M0 and 1/(M0 M1);
- chain start: i / L = umulhi(i, m) >> (s - 1), m = floor(2^(31+s) / L) + 1, s = ceil(log2 L),
  for 0 <= i < 2^25.
"""
import numpy as np
import pytest


def _f32_neighbours(x):
    x = np.float32(x)
    return [np.nextafter(x, np.float32(0)), x, np.nextafter(x, np.float32(np.inf))]


@pytest.mark.parametrize("R", range(1, 8))
def test_stencil_offsets_from_reciprocal_products(R):
    W = 2 * R + 1
    code = np.arange(W ** 3, dtype=np.int32)
    a = code.astype(np.float32) + np.float32(0.5)
    for r1 in _f32_neighbours(1.0 / W):
        for r2 in _f32_neighbours(1.0 / (W * W)):
            q1 = (a * r1).astype(np.int32)          # float32 product, truncated like v_cvt_i32_f32
            q2 = (a * r2).astype(np.int32)
            assert np.array_equal(code - q1 * W, code % W)
            assert np.array_equal(q1 - q2 * W, (code // W) % W)
            assert np.array_equal(q2, code // (W * W))


@pytest.mark.parametrize("M", [(3, 3, 3), (39, 39, 39), (41, 41, 41), (7, 5, 3), (89, 89, 89), (133, 133, 133),
                               (1000, 700, 3), (1290, 1290, 1290)])
def test_cell_coordinates_from_reciprocal_products(M):
    M0, M1, M2 = M
    n = M0 * M1 * M2
    inv0 = 1.0 / M0
    inv01 = 1.0 / (float(M0) * float(M1))
    rng = np.random.default_rng(n)
    # every cell of the small boxes; for the large ones the first and last million and a sample
    if n <= 3_000_000:
        lc = np.arange(n, dtype=np.int64)
    else:
        lc = np.concatenate([np.arange(1_000_000), np.arange(n - 1_000_000, n),
                             rng.integers(0, n, 2_000_000)]).astype(np.int64)
    a = lc.astype(np.float64) + 0.5
    qy = (a * inv0).astype(np.int64)
    qz = (a * inv01).astype(np.int64)
    assert np.array_equal(lc - qy * M0, lc % M0)
    assert np.array_equal(qy - qz * M1, (lc // M0) % M1)
    assert np.array_equal(qz, lc // (M0 * M1))


@pytest.mark.parametrize("L", [4, 5, 7, 300, 1000, 4095, 4096, 4097, 65535, 1 << 20, (1 << 25) - 1])
def test_chain_start_by_multiply_high(L):
    s = 0
    while (1 << s) < L:
        s += 1
    m = (1 << (31 + s)) // L + 1
    assert m < (1 << 32)
    for start in range(0, 1 << 25, 1 << 22):
        i = np.arange(start, start + (1 << 22), dtype=np.uint64)
        q = ((i * np.uint64(m)) >> np.uint64(32)) >> np.uint64(s - 1)
        assert np.array_equal(q, i // np.uint64(L))

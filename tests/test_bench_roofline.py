"""The benchmark's roofline arithmetic, on the CPU: the canonical candidate count of the grid
search, the flop count per launch, and the fractions the bench line reports."""
import math

import pytest

import bench


def test_canonical_candidates_closed_form():
    """27 cells of edge L / floor(L / rc) at the box's mean density: for a cube of 19 cells of
    edge 10.8409 A holding 300,000 atoms in 205.9765^3 A^3 that is 27 * 10.8409^3 * n."""
    L, rc, N = 205.9765, 10.5, 300000
    M = math.floor(L / rc)
    assert M == 19
    expect = 27.0 * (L / M) ** 3 * N / L ** 3
    assert bench.canonical_candidates(N, [L, L, L], rc) == pytest.approx(expect, rel=1e-12)
    assert expect == pytest.approx(1180.93, abs=0.01)
    # orthorhombic: the cell volume is the product of the three edges
    box = [100.0, 60.0, 45.0]
    Ms = [math.floor(x / rc) for x in box]
    cell = (100.0 / Ms[0]) * (60.0 / Ms[1]) * (45.0 / Ms[2])
    assert bench.canonical_candidates(1000, box, rc) == pytest.approx(27 * cell * 1000 / (100 * 60 * 45))


def test_lj_roofline_fields(monkeypatch):
    """achieved = (8 C N + 13 P) / t; frac against 157.3 TF; the stencil-effective figure uses the
    walked candidates instead; no counter record when its source hash does not match."""
    monkeypatch.setattr(bench, "counter_record", lambda name: {})
    N, L, rc = 300000, 205.9765, 10.5
    pairs, cand_stencil, t_ms = 50_000_000, 190_000_000, 0.14
    r = bench.lj_roofline(N, [L, L, L], rc, cand_stencil, pairs, t_ms, 2, 2, 8)
    cand = bench.canonical_candidates(N, [L, L, L], rc) * N
    flop = 8 * cand + 13 * pairs
    assert r["flop_per_launch"] == pytest.approx(flop)
    assert r["achieved"] == pytest.approx(flop / (t_ms * 1e-3) / 1e12, abs=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / 157.3, abs=1e-4)
    assert r["frac_stencil_effective"] == pytest.approx((8 * cand_stencil + 13 * pairs) / (t_ms * 1e-3) / 1e12 / 157.3,
                                                        abs=1e-4)
    assert r["bound"] == "alu" and r["traffic"] is None and "counter_fp32_tflops" not in r


def test_counter_record_follows_the_source(monkeypatch, tmp_path):
    """The committed counter record is used only for the kernel and source it was taken on."""
    rec = tmp_path / "rec.json"
    rec.write_text('{"kernel": "k_lj_tile/R2/K2/H8", "source_sha256": "%s", "bytes_per_launch": 5}'
                   % bench.lj_source_hash())
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(rec))
    assert bench.counter_record("k_lj_tile/R2/K2/H8")["bytes_per_launch"] == 5
    assert bench.counter_record("k_lj_tile/R2/K2/H4") == {}
    rec.write_text('{"kernel": "k_lj_tile/R2/K2/H8", "source_sha256": "0", "bytes_per_launch": 5}')
    assert bench.counter_record("k_lj_tile/R2/K2/H8") == {}


def test_tuning_classes():
    t = bench.tuning_classes([6300, 9900, 120000], [(2, 2, 16), (2, 2, 8), (2, 2, 8)])
    assert t == {"R2/K2/H16": {"boxes": 1, "atoms_min": 6300, "atoms_max": 6300},
                 "R2/K2/H8": {"boxes": 2, "atoms_min": 9900, "atoms_max": 120000}}

"""The counted flops per ECM point behind the benchmark's roofline: the host
count of the device material routine matches the constants the benchmark
uses, and the weighting's count matches a count by hand."""
import shutil

import pytest

from bench import C_CM, C_W


@pytest.mark.skipif(shutil.which('g++') is None, reason="needs a host C++ compiler")
def test_counted_flops_match_bench_constants():
    from paper_2307_16894_amd.flop_count import count
    c = count()
    assert c['material_min'] == C_CM and c['weighting'] == C_W
    # weighting by hand: per tangent column four entries w (a b + c d) (4 ops
    # each) and eight fused multiply-adds into D (16), four columns; then
    # W = w (P F_mu^-T), four entries of a multiply, a fused multiply-add and a
    # multiply (4 each)
    assert C_W == 4 * (4 * 4 + 8 * 2) + 4 * 4
    # the plastic branches cost more than the elastic ones
    assert all(x['material'] > min(y['material'] for y in c['cases']) for x in c['cases'] if x['plastic'])

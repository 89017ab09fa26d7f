"""The flop/byte model reproduces the constants the paper prints (Sec. 2 and
Sec. 4.1), stored with their citations in tests/golden/paper_constants.json."""
import json
import os

from oracle import accounting as A

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_constants.json")))


def test_flop_counts():
    assert A.FLOP_PER_DIRECTION == 168
    assert A.FLOP_HOP_SITE == 1320
    assert A.FLOP_DW_SITE == GOLD["flop_per_site_dw"]["value"]


def test_paper_byte_per_flop():
    b = A.paper_no_reuse_bytes_per_site(real_bytes=4, link_reals=18)
    assert b == 1536
    ratio = b / A.FLOP_DW_SITE
    assert round(ratio, GOLD["byte_per_flop"]["digits"]) == GOLD["byte_per_flop"]["value"]


def test_footprint_16_4():
    g, s = A.footprint_bytes((16, 16, 16, 16), real_bytes=4, link_reals=18)
    fp = GOLD["footprint_16x16x16x16_fp32"]
    assert g == fp["gauge_MiB"] * 2 ** 20
    assert s == fp["spinor_MiB"] * 2 ** 20


def test_ideal_reuse_bytes():
    assert A.hop_bytes_per_output_site("f32", "f32", 18) == 768
    assert A.hop_bytes_per_output_site("f32", "f32", 12) == 576
    assert A.hop_bytes_per_output_site("f64", "f64", 18) == 1536
    assert A.apply_bytes_per_site("f32", "f32", 18) == 816
    assert A.apply_bytes_per_site("f32", "f32", 12) == 624
    assert A.apply_bytes_per_site("bf16", "f16", 12) == 312
    assert A.apply_flop(32 ** 3 * 64) == 1320 * 2097152

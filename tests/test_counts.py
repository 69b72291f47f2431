"""Pin the flop/byte conventions used for GFLOP/s and roofline figures against the
values printed in Table 1 of Sec. 2 (tests/golden/table1.json)."""
import json
import os

from paper_1811_00893_amd import counts

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))


def test_flops_per_site():
    assert counts.HOP_FLOPS_PER_SITE == 1320
    assert counts.FULL_D_FLOPS_PER_SITE == GOLD["wilson"]["flop_per_site"]
    # clover adds two 6x6 Hermitian block mat-vecs (2 x (36 cmul + 30 cadd)) and the add of 24 reals
    clover_extra = 2 * (36 * 6 + 30 * 2) + 24
    assert counts.FULL_D_FLOPS_PER_SITE + clover_extra == GOLD["clover"]["flop_per_site"]


def test_bytes_per_site_and_rooflines():
    w, c = GOLD["wilson"], GOLD["clover"]
    nb = counts.table1_no_reuse_bytes_per_site("fp32")
    assert nb == w["bytes_per_site_float"]
    clover_bytes = nb + 2 * 36 * 4  # two 6x6 Hermitian blocks = 72 floats
    assert clover_bytes == c["bytes_per_site_float"]
    bf = nb / counts.FULL_D_FLOPS_PER_SITE
    assert round(bf, 2) == w["byte_per_flop"]
    assert round(clover_bytes / GOLD["clover"]["flop_per_site"], 2) == c["byte_per_flop"]
    # ideal reuse: each link and vector loaded once
    ideal = counts.full_d_bytes_per_site("fp32")
    assert ideal == 480
    assert round(ideal / counts.FULL_D_FLOPS_PER_SITE, 3) == w["byte_per_flop_ideal"]
    assert round((ideal + 288) / 1944, 3) == c["byte_per_flop_ideal"]
    ito = GOLD["bandwidth_gbs"]["ito_ddr4"]
    assert round(ito / bf) == w["roofline_ito"]
    assert round(ito / (ideal / 1368)) == w["roofline_ito_ideal"]
    assert round(ito / (clover_bytes / 1944)) == c["roofline_ito"]
    assert abs(ito / ((ideal + 288) / 1944) - c["roofline_ito_ideal"]) < 1
    ofp = GOLD["bandwidth_gbs"]["ofp_mcdram_low"]
    assert abs(ofp / bf - w["roofline_ofp"]) < 1.5
    assert abs(ofp / (ideal / 1368) - w["roofline_ofp_ideal"]) < 5


def test_clover_counts():
    c = GOLD["clover"]
    assert counts.CLOVER_FLOPS_PER_SITE == c["flop_per_site"]
    assert counts.table1_no_reuse_bytes_per_site("fp32") + counts.clover_term_bytes("fp32") == c["bytes_per_site_float"]
    ideal = counts.clover_full_bytes_per_site("fp32")
    assert round(ideal / counts.CLOVER_FLOPS_PER_SITE, 3) == c["byte_per_flop_ideal"]
    assert counts.clover_full_bytes_per_site("fp64") == 1536


def test_hop_bytes():
    assert counts.hop_bytes_per_site("fp64") == 1536
    assert counts.hop_bytes_per_site("fp32") == 768
    assert counts.hop_bytes_per_site("fp16") == 392
    assert counts.hop_bytes_per_site("fp16", "fp32") == 680
    assert counts.full_d_bytes_per_site("fp64") == 960
    assert counts.bicgstab_iter_bytes_per_even_site("fp64") == 9408

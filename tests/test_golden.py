"""The paper's stated per-site counts, recomputed from the stencil's structure.

The single-right-hand-side Dslash moves, per lattice site, 16 neighbour vectors
(6 reals) and 16 links (18 reals) plus the 6-real result, and does 16 complex
3x3 matrix-vector products accumulated into one vector plus an axpy-type update
(Sec. 6.2).  These counts are what the byte model of the bench is built on.
"""
import json
import os

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def load():
    with open(GOLDEN) as f:
        return json.load(f)


def test_dslash_counts():
    g = load()["dslash_single_rhs_per_site"]
    n = g["neighbours"]
    words = n * (g["reals_per_vector"] + g["reals_per_link"]) + g["reals_per_vector"]
    assert words == g["words"]
    cmatvec = 9 * 6 + 6 * 2            # 9 complex multiplies, 6 complex adds
    flops = n * cmatvec + (n - 1) * 6 + 12   # accumulate 16 results, then a x + y
    assert flops == g["flops"]
    ai = flops / (words * 4)
    assert abs(ai - g["arithmetic_intensity_single"]) < 0.005


def test_block_sizes_cover_total():
    g = load()["block_sizes"]
    for nb in g["value"]:
        assert g["total_rhs"] % nb == 0
    assert max(g["value"]) == load()["max_block_size"]["value"]

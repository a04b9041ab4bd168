"""The Vamana pins must catch plausible mistakes in the oracle's build.

Each case plants one mistake in a copy of oracle/dpc_oracle.c (on the CPU, in a
temporary directory), builds it, points the oracle module at the copy and runs
the pins of tests/test_vamana_pins.py: at least one must fail.  The mistakes:
searching the live graph instead of the batch-start snapshot, leaving Nout(p)
out of the forward candidates, appending reverse edges already present, pruning
the first pass with alpha instead of 1, ramping the second pass's batches,
skipping the first point in the second pass, doubling batches past the cap,
keeping the earliest instead of the closest visited points under a cap, and a
wrong start set.
"""
import os
import subprocess

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "dpc_oracle.c")

MUTATIONS = {
    "live_graph": [
        ("#pragma omp parallel for schedule(dynamic, 1)\n      for (int64_t t = 0; t < nb; ++t) {",
         "for (int64_t t = 0; t < nb; ++t) {"),
        ("          new_deg[t] = no < 0 ? 0 : no;\n",
         "          new_deg[t] = no < 0 ? 0 : no;\n"
         "          for (int32_t e = 0; e < R; ++e)\n"
         "            adj[p * R + e] = e < new_deg[t] ? (int32_t)new_out[t * R + e] : -1;\n"
         "          deg[p] = new_deg[t];\n")],
    "drop_nout": [("          for (int32_t e = 0; e < deg[p]; ++e) myvis[nvis++] = adj[p * R + e];\n", "")],
    "duplicate_reverse_edges": [
        ("for (int32_t u = 0; u < nold; ++u) if (tmp[u] == edges[e].src) { present = 1; break; }", "")],
    "pass1_alpha": [("const double a = (passes > 1 && pass == 0) ? 1.0 : alpha;", "const double a = alpha;")],
    "pass2_ramped_batches": [("int64_t bsize = pass == 0 ? 1 : cap;", "int64_t bsize = 1;")],
    "pass2_skips_first_point": [("int64_t inserted = pass == 0 ? 1 : 0;", "int64_t inserted = 1;")],
    "doubling_past_cap": [("if (bsize < cap) bsize *= 2;", "")],
    "visited_cap_keeps_earliest": [("qsort(cv, (size_t)nvis, sizeof(cand_t), cmp_cand);", "")],
    "single_start": [("int32_t ns = (int32_t)(in_graph < num_starts ? in_graph : num_starts);",
                      "int32_t ns = (int32_t)(in_graph < 1 ? in_graph : 1);")],
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_pins_catch_mutation(name, tmp_path):
    import test_vamana_pins as pins
    s = open(SRC).read()
    for a, b in MUTATIONS[name]:
        assert a in s, f"mutation site of {name} not found in the oracle source"
        s = s.replace(a, b)
    c = tmp_path / "mut.c"
    so = tmp_path / "libmut.so"
    c.write_text(s)
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", str(so), str(c),
                    "-lm"], check=True)
    saved = (oracle._LIB, oracle._lib)
    oracle._LIB, oracle._lib = str(so), None
    failed = []
    try:
        for t in sorted(x for x in dir(pins) if x.startswith("test_")):
            try:
                getattr(pins, t)(None)
            except AssertionError:
                failed.append(t)
    finally:
        oracle._LIB, oracle._lib = saved
    assert failed, f"no pin caught the mistake {name}"

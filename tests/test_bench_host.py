"""Host logic of bench.py (no GPU): the kernel-source hash that decides
whether a committed counter summary still describes the current code, and
the counts the roofline line is built from."""
import os
import shutil

import numpy as np

import bench


def test_code_text_drops_comments_and_whitespace_only():
    src = ('int a = 1; // a comment with a quote \' and "\n'
           '/* block\n comment */ const char *s = "a // b /* c */";\n'
           "char q = '/'; char e = '\\''; x = y / z;\n")
    assert bench.code_text(src) == ('inta=1;constchar*s="a // b /* c */";'
                                    "charq='/';chare='\\'';x=y/z;")


def test_source_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    root = tmp_path / "repo"
    csrc = root / "paper_1907_04034_amd" / "csrc"
    shutil.copytree(os.path.join(bench.ROOT, "paper_1907_04034_amd", "csrc"), csrc)
    monkeypatch.setattr(bench, "ROOT", str(root))
    base = bench.source_hash()
    f = csrc / "pairs.hip"
    text = f.read_text()
    f.write_text("// a new comment line\n" + text.replace("\n", "\n  ", 3))
    assert bench.source_hash() == base
    f.write_text(text.replace("+ 1", "+ 2", 1))
    assert bench.source_hash() != base


def test_committed_counter_summaries_match_the_kernel_sources():
    # the roofline's traffic and bound come from these only while they
    # describe the current code
    for prec in ("fp64", "fp32"):
        got = bench.counters_summary("C5", prec)
        assert got is not None and got["traffic"] > 0 and got["bound"] in ("hbm", "alu")


def test_force_bytes_counts_records_in_3d_and_fields_in_2d_fp64():
    n = 1000
    types = np.zeros(n, dtype=np.int8)
    counts = np.full(n, 30)
    b3 = bench.force_bytes(counts, types, 8, 3)
    # 3D FP64: a 96-byte record per row, the row's own fields and table
    own = 8 * 3 + 2 * 8 * 3 + 3 * 8 + 4
    assert b3 == n * (1 + 96) + n * own + 4 * 30 * n + n * (2 * 8 * 3 + 2 * 8)
    b2 = bench.force_bytes(counts, types, 8, 2)
    nbr2 = 8 * 2 + 2 * 8 * 2 + 2 * 8 + 1
    own2 = 8 * 2 + 2 * 8 * 2 + 3 * 8 + 4
    assert b2 == n * (1 + nbr2) + n * own2 + 4 * 30 * n + n * (2 * 8 * 2 + 2 * 8)

"""Host logic of bench.py that needs no GPU: the source fingerprint that ties
the recorded HBM traffic counters to the kernel code they were taken on."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_code_only_drops_comments_and_blank_lines():
    src = ('// file comment\n#include "a.h"  // trailing\n\n/* block\n comment */\n'
           'int f() { return 1; }   \n')
    assert bench._code_only(src) == '#include "a.h"\nint f() { return 1; }'


def test_code_only_keeps_literals_that_look_like_comments():
    src = 'const char *s = "http://x /* y */";\nchar c = \'/\';  // c\n'
    assert bench._code_only(src) == 'const char *s = "http://x /* y */";\nchar c = \'/\';'


def test_fingerprint_ignores_comment_edits_but_not_code_edits(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_1011_0093_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in bench._KERNEL_SOURCES:
        (csrc / name).write_text("// v1\nint x = 1;\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_sources_hash()
    (csrc / bench._KERNEL_SOURCES[0]).write_text("// another comment\n\nint x = 1;  // same code\n")
    assert bench.kernel_sources_hash() == h0
    (csrc / bench._KERNEL_SOURCES[0]).write_text("int x = 2;\n")
    assert bench.kernel_sources_hash() != h0


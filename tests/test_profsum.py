"""The profile summariser's source hash: comments do not count, code does."""
import os

from paper_1307_1955_amd import profsum

SRC = '''// leading comment
#include "x.h"
/* a block
   comment */ int f(int a) {   // trailing
    const char* s = "not // a comment /* nor this */";
    char q = '"';  /* q */ char e = '\\\\';
    return a + 1;
}
'''


def test_code_only_drops_comments_and_keeps_literals():
    got = profsum.code_only(SRC)
    assert got.splitlines() == ['#include "x.h"', 'int f(int a) {',
                                'const char* s = "not // a comment /* nor this */";',
                                "char q = '\"'; char e = '\\\\';", "return a + 1;", "}"]


def test_comment_edits_keep_code_changes_break():
    base = profsum.code_only(SRC)
    assert profsum.code_only(SRC.replace("// trailing", "// another remark")) == base
    assert profsum.code_only(SRC.replace("a block", "a reworded block")) == base
    assert profsum.code_only(SRC.replace("    return", "\n\n        return")) == base
    assert profsum.code_only(SRC.replace("a + 1", "a + 2")) != base
    assert profsum.code_only(SRC.replace("nor this", "nor that")) != base


def test_sources_hash_reads_every_kernel_source():
    for rel in profsum.KERNEL_SOURCES:
        assert os.path.exists(os.path.join(profsum.PKG, rel)), rel
    h = profsum.sources_hash()
    assert len(h) == 64 and int(h, 16) >= 0

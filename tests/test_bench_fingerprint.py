"""bench.py keys its recorded HBM traffic to a fingerprint of the ray
kernels' code.  The fingerprint drops comments (a comment edit does not
change the kernel) but keeps every token of code, string literals included."""
import bench


def test_comments_and_whitespace_do_not_count():
    a = "int a = 1; // one\n/* a\n block */ float b;\n"
    b = "int a = 1;\n\n   float   b; // changed comment\n"
    assert bench.code_text(a) == bench.code_text(b) == "int a = 1; float b;"


def test_code_and_strings_count():
    assert bench.code_text("int a = 1;") != bench.code_text("int a = 2;")
    s = 'const char *p = "x // y"; /* c */'
    assert bench.code_text(s) == 'const char *p = "x // y";'
    assert bench.code_text('f("/* q */");') == 'f("/* q */");'


def test_fingerprint_is_stable():
    assert bench.source_sha() == bench.source_sha()
    assert len(bench.source_sha()) == 16

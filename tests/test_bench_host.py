"""Host logic of bench.py that needs no GPU."""
import bench


def test_code_text_drops_comments_and_layout():
    a = "int f(int x) {\n  // comment\n  return x /* inline */ + 1;\n}\n"
    b = "int f(int x) { return x + 1; } // a different comment\n"
    assert bench.code_text(a) == bench.code_text(b) == "int f(int x) { return x + 1; }"


def test_code_text_keeps_strings_and_code_changes():
    s = 'const char* m = "a // b /* c */"; char q = \'"\'; x = "\\"//";'
    assert bench.code_text(s) == s
    assert bench.code_text("return x + 1;") != bench.code_text("return x + 2;")


def test_kernel_hash_is_stable():
    assert bench.kernel_hash() == bench.kernel_hash()
    assert len(bench.kernel_hash()) == 16

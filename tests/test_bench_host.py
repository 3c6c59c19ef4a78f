"""CPU tests of bench.py's host logic: the stage-source fingerprint that ties
the committed counter summaries to the kernel code ignores comments and
layout but not code, and counter summaries for other code are refused."""
import os

import bench


def test_code_text_drops_comments_and_layout_but_keeps_literals():
    src = ('int a = 1; // trailing\n/* block\n comment */ int  b =\t2;\n'
           'const char* s = "// kept"; const char* t = "/* kept */"; char q = \'"\'; char e = \'\\\'\';\n')
    assert bench._cxx_code(src) == ('int a = 1; int b = 2; const char* s = "// kept"; '
                                    'const char* t = "/* kept */"; char q = \'"\'; char e = \'\\\'\';')


def test_code_text_separates_tokens_a_comment_separated():
    # a block comment between two tokens leaves them two tokens
    assert bench._cxx_code("a/**/b") == "a b"
    assert bench._cxx_code("x - -y") != bench._cxx_code("x --y")


def test_fingerprint_follows_code_not_comments(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    build = tmp_path / "build.py"
    build.write_text("FLAGS = ['-O3']\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "STAGE_SOURCES", ("k.hip", "build.py"))
    src.write_text("// version one\n__global__ void k(double* x) { x[0] = 1.0; }\n")
    h0 = bench.stage_source_hash()
    src.write_text("/* reworded */\n__global__ void k(double* x) {\n  x[0] = 1.0;  // same code\n}\n")
    assert bench.stage_source_hash() == h0
    src.write_text("__global__ void k(double* x) { x[0] = 2.0; }\n")
    assert bench.stage_source_hash() != h0
    src.write_text("__global__ void k(double* x) { x[0] = 1.0; }\n")
    build.write_text("FLAGS = ['-O2']\n")
    assert bench.stage_source_hash() != h0


def test_counter_summaries_for_other_code_are_refused(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "STAGE_SOURCES", ("k.hip",))
    (tmp_path / "k.hip").write_text("__global__ void k() {}\n")
    os.makedirs(tmp_path / "profiles")
    (tmp_path / bench.TRAFFIC_FILE).write_text(
        "source_hash = 0000000000000000\nn = 360\norder = 5\nscheme = weno\nlaunch = 30,3\n"
        "fetch_bytes = 1\nwrite_bytes = 1\nbytes_per_launch = 2\ncopy_factor_fetch = 1\ncopy_factor_write = 1\n")
    assert bench.measured_traffic(360, 5, "weno", (30, 3)) is None
    text = (tmp_path / bench.TRAFFIC_FILE).read_text().replace("0000000000000000", bench.stage_source_hash())
    (tmp_path / bench.TRAFFIC_FILE).write_text(text)
    got = bench.measured_traffic(360, 5, "weno", (30, 3))
    assert got is not None and got["bytes_per_launch"] == 2.0
    assert bench.measured_traffic(360, 5, "weno", (60, 3)) is None

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


def test_workload_line_shape():
    class Args:
        steps, warmup = 3, 1
    roof = {"bound": "hbm", "frac": 0.5}
    def run(v):
        return {"value": v, "ms_per_step": 1.0, "schedule": {"steps_per_pass": 5},
                "roofline": roof, "norm_drift": 0.0}
    line = bench.workload_line({"c64": run(2.0), "c128": run(1.0)}, Args, "w", (8, 4), 10, 0.1,
                               boundary="closed")
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline"):
        assert key in line
    assert line["dtype"] == "c64" and line["value"] == 2.0
    assert line["config"] == {"workload": "w", "mesh": [8, 4], "time_steps_per_solve": 10,
                              "dt": 0.1, "boundary": "closed", "steps_per_pass": 5}
    assert line["complex128"]["value"] == 1.0
    only = bench.workload_line({"c128": run(1.5)}, Args, "w", (8, 4), 10, 0.1)
    assert only["dtype"] == "c128" and "complex64" not in only and "complex128" not in only


def test_3d_hash_covers_its_own_sources():
    """The 3D counters are keyed by the code of the 3D march and of the 2D headers it
    includes: a different key from the 2D one, stable across calls."""
    assert set(bench.KERNEL_SOURCES[:2]) <= set(bench.KERNEL3_SOURCES)
    h3 = bench.kernel_hash(bench.KERNEL3_SOURCES)
    assert h3 == bench.kernel_hash(bench.KERNEL3_SOURCES) != bench.kernel_hash()
    assert len(h3) == 16

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
                "roofline": roof, "precision": {"norm_drift": 0.0}}
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


def test_roofline_uses_three_working_dtype_elements_per_site():
    """frac = (read psi + write psi + read phase, each in the working dtype) per site
    of one pass over the average launch time, against 8 TB/s."""
    for dtype, per_site in (("c64", 24), ("c128", 48)):
        r = bench.roofline(dtype, 1000, 1e-6, 1e9, None)
        assert r["algorithmic_bytes_per_site"] == per_site
        assert r["algorithmic_bytes_per_launch"] == 1000 * per_site
        assert abs(r["frac"] - 1000 * per_site / 1e-6 / 8e12) < 1e-4
        assert r["table_extra_bytes_per_launch"] == 0
        assert r["traffic"] is None and "traffic_frac" not in r
    r = bench.roofline("c64", 1000, 1e-6, 1e9, 30000.0)
    assert r["traffic_over_algorithmic"] == 1.25


def test_vs_oracle_differences():
    ref = {"norm_start": 1.0, "norm_end": 1.0 - 1e-15, "energy_start": 2.0, "energy_end": 2.5}
    got = {"norm_start": 1.0, "norm_end": 1.0 + 1e-8, "energy_start": 2.0, "energy_end": 2.5005}
    v = bench.vs_oracle(got, ref)
    assert abs(v["energy_end_rel_diff"] - 2e-4) < 1e-12
    assert v["energy_start_rel_diff"] == 0.0
    assert abs(v["oracle_energy_drift"] - 0.5) < 1e-15
    assert abs(v["norm_end_minus_oracle"] - (1e-8 + 1e-15)) < 1e-15


def test_oracle_observables_fixture():
    """The committed oracle norm and energy of the 4096^2 workload: both starting
    states normalised (the complex64 one to its rounding), the oracle's norm
    conserved to 1e-13 and its energy drift the second-order O(dt^2) size."""
    import json
    with open(bench.ORACLE_OBSERVABLES) as f:
        d = json.load(f)
    assert d["steps"] == 1000 and d["mesh"] == [4096, 4096]
    for name in ("c128", "c64"):
        r = d["inputs"][name]
        assert abs(r["norm_start"] - 1.0) < (1e-12 if name == "c128" else 1e-6)
        assert abs(r["norm_end"] - r["norm_start"]) < 1e-13
        assert 0 < abs(r["energy_end"] - r["energy_start"]) < 1e-4

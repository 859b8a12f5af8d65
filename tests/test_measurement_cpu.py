"""Host-side checks of the measurement plumbing (no GPU): the benchmark refuses more than one GPU,
and the rocprofv3 summaries scale the HBM counters by the calibration copy and tie the traffic to
the sources it was measured on."""
import json
import os
import sqlite3
import subprocess
import sys

from paper_1702_03154_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

KIB = float(1 << 20)   # the 1 GiB calibration copy in KiB


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _counter_db(path, rows):
    c = sqlite3.connect(path)
    c.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
              "value real)")
    c.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    c.commit()
    c.close()


def _runs(tmp_path):
    """A FETCH_SIZE and a WRITE_SIZE run: a small runtime copy, the calibration copy (which the
    counters read as half its bytes fetched and all of them written), a build kernel, two lookups."""
    lib = "mphfk::(anonymous namespace)::"
    kernels = [(1, "__amd_rocclr_copyBuffer", 4.0, 4.0),
               (2, "__amd_rocclr_copyBuffer", KIB / 2, KIB),
               (3, lib + "k_bucket<true>(unsigned long const*)", 100.0, 50.0),
               (4, lib + "k_lookup(unsigned long const*)", 1000.0, 300.0),
               (5, lib + "k_lookup(unsigned long const*)", 1200.0, 300.0)]
    f, w = str(tmp_path / "fetch.db"), str(tmp_path / "write.db")
    _counter_db(f, [(d, n, "FETCH_SIZE", fv) for d, n, fv, _ in kernels])
    _counter_db(w, [(d, n, "WRITE_SIZE", wv) for d, n, _, wv in kernels])
    return f, w


def test_lookup_traffic_is_scaled_by_the_calibration_copy(tmp_path):
    f, w = _runs(tmp_path)
    out = str(tmp_path / "t.json")
    profsum.traffic(f, w, "k_lookup", 10**6, out)
    t = json.load(open(out))
    assert t["fetch_scale"] == 2.0 and t["write_scale"] == 1.0
    assert t["fetch_kib"] == 1100.0 and t["write_kib"] == 300.0   # mean over the launches
    assert t["bytes_per_launch"] == (1100.0 * 2.0 + 300.0) * 1024.0
    assert t["source_sha256"] == profsum.source_digest()


def test_build_traffic_counts_library_kernels_before_the_first_lookup(tmp_path):
    f, w = _runs(tmp_path)
    out = str(tmp_path / "b.json")
    profsum.build_traffic(f, w, 10**6, out)
    t = json.load(open(out))
    assert t["fetch_kib"] == 100.0 and t["write_kib"] == 50.0
    assert t["bytes_per_build"] == (100.0 * 2.0 + 50.0) * 1024.0
    assert t["source_sha256"] == profsum.source_digest(profsum.BUILD_SOURCES)
    assert t["source_sha256"] != profsum.source_digest()


def test_short_names_drop_namespace_and_arguments():
    assert profsum.short("mphfk::(anonymous namespace)::k_lookup(unsigned long const*, int)") == "k_lookup"
    assert profsum.short("void mphfk::(anonymous namespace)::k_bucket<true>(int)") == "void k_bucket<true>"


def test_steps_split_a_trace_into_build_and_lookup(tmp_path):
    """profsum steps: each step ends with a k_lookup dispatch; its build is every library kernel since
    the previous one (torch kernels and the roofline probes left out)."""
    import io
    import sqlite3

    db = str(tmp_path / "k.db")
    c = sqlite3.connect(db)
    c.execute("create table kernels(name text, start int, end int, grid_x int, workgroup_x int)")
    rows = [("void at::native::fill_kernel(int)", 0, 10, 1, 1),
            ("void mphfk::(anonymous namespace)::k_partition<8, false, false, 3>(x)", 100, 1100, 10, 768),
            ("mphfk::(anonymous namespace)::k_bucket<true>(x)", 1200, 1700, 10, 1024),
            ("mphfk::(anonymous namespace)::k_lookup(x)", 2000, 3000, 4096, 256),
            ("(anonymous namespace)::k_probe_copy(x)", 3100, 3200, 1, 1),
            ("mphfk::(anonymous namespace)::k_tail(x)", 4000, 4300, 1, 1024),
            ("mphfk::(anonymous namespace)::k_lookup(x)", 5000, 7000, 4096, 256)]
    c.executemany("insert into kernels values (?,?,?,?,?)", rows)
    c.commit()
    out = io.StringIO()
    profsum.steps(db, 5, out)
    lines = out.getvalue().splitlines()
    # step 0: two build kernels, 1.5 us busy over a 1.6 us span; step 1: the tail only
    assert lines[1].split()[:5] == ["0", "2", "0.002", "0.002", "0.001"]
    assert lines[2].split()[:5] == ["1", "1", "0.000", "0.000", "0.002"]
    assert "mean k_lookup over steps 1..1" in lines[3] and lines[3].endswith("0.002 ms")
    assert any(l.startswith("k_tail") for l in lines[5:])
    assert not any("k_probe" in l for l in lines)
    assert profsum.short("(anonymous namespace)::k_probe_copy(x)") == "k_probe_copy"

"""Host helpers of bench.py (no GPU): the traffic summary lookup and the plan names."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_lookup(tmp_path):
    b = load_bench()
    f = tmp_path / "t.txt"
    f.write_text("# comment\nsource_hash: abc\nbytes_per_launch[table-split-n1=8:fwd_row]: 146540105\n")
    assert b.read_traffic("table-split-n1=8:fwd_row", "abc", str(f)) == 146540105.0
    assert b.read_traffic("table-split-n1=8:inv_row", "abc", str(f)) is None
    assert b.read_traffic("table-split-n1=8:fwd_row", "other", str(f)) is None   # stale counters
    f.write_text("source_hash: abc\nvalu_insts_per_launch[table-split-n1=6:inv_row]: 11554560\n")
    assert b.read_traffic("table-split-n1=6:inv_row", "abc", str(f), field="valu_insts_per_launch") == 11554560.0
    assert b.read_traffic("table-split-n1=6:inv_row", "abc", str(f)) is None


def test_committed_traffic_covers_its_configuration():
    b = load_bench()
    path = os.path.join(ROOT, "profiles", "traffic_counters.txt")
    text = open(path).read()
    h = [l.split(":", 1)[1].strip() for l in text.splitlines() if l.startswith("source_hash")][0]
    keys = [l.split("]")[0].split("[", 1)[1] for l in text.splitlines() if l.startswith("bytes_per_launch[")]
    assert keys
    for k in keys:
        assert b.read_traffic(k, h) > 0
    # the plans that win the headline measurement on some box (the default split and the tuner's)
    # carry bytes and instruction counts for all four passes
    plans = {k.split(":")[0] for k in keys} | {"table-split-n1=6", "table-split-n1=8"}
    for plan in plans:
        for kern in ("fwd_col", "fwd_row", "inv_row", "inv_col"):
            assert b.read_traffic(f"{plan}:{kern}", h) > 0
            assert b.read_traffic(f"{plan}:{kern}", h, field="valu_insts_per_launch") > 0


def test_plan_names():
    b = load_bench()
    assert b.variant_key({"kernel_path": 1, "log2_n1": 8}, 0) == "table-split-n1=8"
    assert b.variant_key({"kernel_path": 2, "log2_n1": 7}, 2) == "ot2-fused-n1=7"
    assert b.variant_key({"kernel_path": 1, "log2_n1": 6, "r1": 4, "wg_size": 0, "col_width": 32}, 1) == \
        "ot1-split-n1=6-r1=4-col_width=32"


def test_bench_refuses_several_gpus():
    """The measurement covers one GPU: --gpus above 1 exits with status 2 and says why, before
    touching any device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "single MI355X" in r.stderr and r.stdout == ""

"""bench.py's contract on the host: more than one GPU is refused with a message
before anything touches a device, and the kernel-source hash keying the traffic
record covers the generate tile kernels' sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 1" in r.stderr


def test_traffic_record_is_keyed_by_the_generate_kernel_sources():
    import json

    import bench
    h = bench.kernel_source_hash()
    assert len(h) == 16
    for f in bench.DEVICE_SOURCES:
        assert os.path.exists(os.path.join(ROOT, "paper_1811_11629_amd", "csrc", f)), f
    rec = json.load(open(os.path.join(ROOT, "profiles", "tile_kernel_traffic.json")))
    ent = rec["multi_instance_e3"]
    # the record names its kernel and carries both counter passes and the copy calibration
    for k in ("kernel", "kernel_source_hash", "fetch_size_kib", "write_size_kib",
              "copy_fetch_factor", "copy_write_factor", "hbm_bytes_per_launch"):
        assert k in ent, k
    # other shapes measured on the same sources carry their own two passes
    for o in ent.get("other_kernels", []):
        for k in ("kernel", "command", "fetch_size_kib", "write_size_kib", "hbm_bytes_per_launch"):
            assert k in o, k


def test_source_hash_ignores_comments_and_layout_only():
    import bench
    base = "int f(int x) {\n  return x + 1;  // one\n}\n/* note */\nconst char* s = \"a // b\";\n"
    same = "int f(int x) { return x + 1; }\n// other words\nconst char* s = \"a // b\"; /* x */\n"
    assert bench.code_only(base) == bench.code_only(same)
    # a changed operator, constant or string literal changes the code
    for changed in (base.replace("x + 1", "x - 1"), base.replace("1;", "2;"),
                    base.replace("a // b", "a / b")):
        assert bench.code_only(changed) != bench.code_only(base)
    # comment markers inside literals are code, and an escaped quote stays inside its literal
    assert bench.code_only('char c = \'"\'; // x\nint y;') == "char c = '\"'; int y;"
    assert bench.code_only('const char* t = "q\\"// not a comment";') == \
        'const char* t = "q\\"// not a comment";'

"""The benchmark's command-line contract, on the CPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_algorithmic_bytes_count_the_layouts_own_index_width():
    """Panels store 2-byte panel-local columns, CSR 4-byte ones, one per B rows
    of a block row; the CSR-equivalent figure always charges 4 bytes.  The
    full-scale FP32 dose with the objective epilogue: nnz*6 + 8(n_vox+1) +
    4(n_bl+n_vox) + 5 n_vox."""
    from types import SimpleNamespace
    b = _bench_module()
    n_vox, n_bl, nnz = 2097152, 288000, 496216960
    info = SimpleNamespace(n_vox=n_vox, n_bl=n_bl, nnz=nnz, value_bytes=4, dose_layout=1, price_layout=1,
                           dose_block_rows=1, price_block_rows=1)
    ab = b.algorithmic_bytes(info)
    assert ab["dose"] == nnz * 6 + 8 * (n_vox + 1) + 4 * (n_bl + n_vox) + 5 * n_vox
    assert ab["price"] == nnz * 6 + 8 * (n_bl + 1) + 4 * (n_vox + n_bl)
    assert abs(ab["dose"] / 1e9 - 3.014) < 1e-3
    csr = b.algorithmic_bytes(info, csr_equivalent=True)
    assert csr["dose"] - ab["dose"] == 2 * nnz
    # 16-bit values, two rows per block row in panels (index 1 byte per value), CSR price with B = 2
    info16 = SimpleNamespace(n_vox=n_vox, n_bl=n_bl, nnz=nnz, value_bytes=2, dose_layout=1, price_layout=0,
                             dose_block_rows=2, price_block_rows=2)
    assert b.index_bytes(info16, "dose") == 1.0 and b.index_bytes(info16, "price") == 2.0
    d16, p16 = b.plain_bytes(info16, 8)
    assert d16 == nnz * 3 + 8 * (n_vox + 1) + 32 * (n_bl + n_vox) + 4 * n_bl
    assert p16 == nnz * 4 + 8 * (n_bl + 1) + 32 * (n_vox + n_bl) + 4 * n_bl
    assert not b.check_peak("test", 8001.0) and b.check_peak("test", 7999.0)


def test_source_hash_ignores_comments_only():
    """The counters' validity key: comments and white-space layout do not
    change it, code does; string and character literals stay whole."""
    from paper_1503_01721_amd.profiling import code_only
    a = 'int a = 1; // one\n/* block "x" */ const char* s = "// kept"; char q = \'/\';\n'
    b = 'int   a = 1;\n\n// another comment\nconst char* s = "// kept"; /* c */ char q = \'/\';'
    assert code_only(a) == code_only(b) == 'int a = 1; const char* s = "// kept"; char q = \'/\';'
    assert code_only("int a = 1;") != code_only("int a = 2;")
    assert code_only('x = "a\\"b // c"; y;') == 'x = "a\\"b // c"; y;'


def test_cpu_baseline_repeats_the_oracle_pairs_to_its_time_floor():
    """The oracle leg: at least one dose + price pair, more until min_seconds
    of host work, never more than max_pairs; the rate counts every pair."""
    b = _bench_module()
    from paper_1503_01721_amd import synth
    plan = synth.PLANS["small_cp8_bl6x6_vox16"]
    d = synth.generate_ddc(plan)
    one = b.cpu_baseline(d, plan, 1e12, 1e12, min_seconds=0.0)
    assert one["sample"].startswith("1 pair of") and one["kind"] == "oracle" and one["cores"] == 1
    two = b.cpu_baseline(d, plan, 1e12, 1e12, min_seconds=1e9, max_pairs=2)
    assert two["sample"].startswith("2 pairs of") and two["value"] > 0 and two["seconds"] > 0


def test_committed_traffic_matches_the_product_code():
    """The HBM counters committed for the benchmark's kernels were taken on the
    product code as it stands (comments aside), so the benchmark reports them."""
    b = _bench_module()
    for kernel in ("dose", "price"):
        for storage in ("f32", "f16"):
            v = b.read_traffic(kernel, "cp180_bl40x40_vox128", storage, "sliced")
            assert v is not None and v > 1e9, (kernel, storage)

"""Host-side checks of the benchmark's byte and op models and of its traffic lookup (no GPU)."""
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_row_kernel_bytes_for_the_benchmarked_launch():
    # N = 2^16 as 64 x 32 x 32, 24 limbs x 16 polynomials, counted term by term:
    # data 24 * 16 * 65536 words read and written; per prime one 128 x 128-byte BAT
    # table (C1 = C2 = 32, 4 x 4 bytes per entry) and 1024 inner twiddle pairs;
    # inverse launches add 65536 step-2 twiddle pairs per prime
    data = 2 * 4 * 24 * 16 * 65536
    per_prime = 128 * 128 + 1024 * 8
    inverse_twiddles = 24 * 65536 * 8
    expect = data + 24 * per_prime + inverse_twiddles // 2
    assert expect == 208207872
    assert bench.rows_bytes_per_launch(16, 6, 5, 24, 16) == expect


def test_row_kernel_bytes_with_unequal_factors():
    # C1 != C2 stages both tables
    got = bench.rows_bytes_per_launch(15, 6, 4, 2, 3)
    n, c1, c2 = 1 << 15, 16, 32
    assert got == 2 * 3 * n * 8 + 2 * (16 * c1 * c1 + 16 * c2 * c2 + 8 * 512) + 2 * n * 8 // 2


def test_counted_traffic_is_close_to_the_model():
    # the committed rocprofv3 counters of the row kernels (average of the forward and the
    # inverse launch): at most 10% above the algorithmic bytes -- the forward is within 1%,
    # the inverse fetches part of its step-2 twiddle pairs more than once (144 MB read
    # against 114 MB)
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
        rec = json.load(f)["ntt_rows"]
    model = bench.rows_bytes_per_launch(16, 6, 5, 24, 16)
    assert model <= rec["bytes_per_launch"] <= 1.10 * model
    assert rec["fetch_bytes"] + rec["write_bytes"] == rec["bytes_per_launch"]


def test_gemm_ops_model():
    # one BAT GEMM step: 2 ops per int8 MAC, (4U)^2 MACs per output column block of V
    assert bench.gemm_ops_per_launch(16, 6, 384, "left") == 2.0 * 256 * 256 * 1024 * 384
    assert bench.gemm_ops_per_launch(12, 6, 1, "right") == 2.0 * 256 * 256 * 64


def test_traffic_is_null_once_the_kernel_changed():
    assert bench.traffic_for("ntt_rows", "0" * 16) is None
    assert bench.traffic_for("no_such_kernel", bench.source_hash("ntt_rows.hip")) is None


def test_he_mult_model_counts_config3():
    # N = 2^16, L = 24, K = 8, dnum = 3 (alpha = 8): INTT(d2) 24 + ModUp 3 x 24 + ModDown 2 x (8 + 24)
    m = bench.he_mult_model(16, 24, 8, 3, 1, 6, 5)
    assert m["limb_ntts"] == 160
    n = 1 << 16
    per_ntt = 32.0 * n * (64 + 32 + 32)
    bconv = 3 * 2.0 * 32 * 96 * n + 2 * 2.0 * 32 * 96 * n
    assert m["int8_ops"] == 160 * per_ntt + bconv
    ct = 2 * 24 * n * 4
    assert m["hbm_bytes"] == 3 * ct + 3 * 2 * 32 * n * 4          # batch 1: the key once per op
    assert bench.he_mult_model(16, 24, 8, 3, 8, 6, 5)["hbm_bytes"] == 3 * ct + 3 * 2 * 32 * n * 4 / 8
    # two factors, 256 x 256: 32 N (R + C) per limb-NTT
    assert bench.he_mult_model(16, 24, 8, 3, 1, 8, 0)["int8_ops"] == 160 * 32.0 * n * 512 + bconv


def test_more_than_one_gpu_is_refused_with_a_message():
    # the bench measures one GPU: --gpus above 1 (or a multi-rank launch) exits before
    # anything touches the device, with a message that says why
    import subprocess
    import sys
    for argv, env in ((["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "4"})):
        r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, cwd=ROOT,
                           env=dict(os.environ, **env), capture_output=True, text=True, timeout=120)
        assert r.returncode == 2
        assert "one GPU only" in r.stderr
        assert r.stdout == ""

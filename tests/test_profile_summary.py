"""Host logic of the traffic figure: the counter summary read from rocprofv3
databases (synthetic ones here, with the tables and columns the summary queries)
and bench.py's use of the committed summary."""
import json
import sqlite3

import pytest

from paper_2507_05222_amd import profile_summary as PS

GEMM32 = "void (anonymous namespace)::k_gemm_jobs<0, 32>((anonymous namespace)::GemmBatch)"
GEMM64 = "void (anonymous namespace)::k_gemm_jobs<0, 64>((anonymous namespace)::GemmBatch)"
GEMM_F32 = "void (anonymous namespace)::k_gemm_jobs<1, 32>((anonymous namespace)::GemmBatch)"


def _pmc_db(path, rows):
    c = sqlite3.connect(path)
    c.execute("create table pmc_events (name text, counter_name text, counter_value real)")
    c.executemany("insert into pmc_events values (?, ?, ?)", rows)
    c.commit()
    c.close()
    return str(path)


def _trace_db(path, rows):
    c = sqlite3.connect(path)
    c.execute("create table kernels (name text, start integer, end integer)")
    c.executemany("insert into kernels values (?, ?, ?)", rows)
    c.commit()
    c.close()
    return str(path)


def test_counter_selects_the_fp64_gemm_class(tmp_path):
    db = _pmc_db(tmp_path / "f.db", [
        (GEMM32, "FETCH_SIZE", 100.0), (GEMM64, "FETCH_SIZE", 300.0),
        (GEMM_F32, "FETCH_SIZE", 1e6),             # another precision class: excluded
        (GEMM32, "WRITE_SIZE", 7.0),               # another counter: excluded
        ("k_cg_step(SBatch, SGeo, SLay)", "FETCH_SIZE", 1e6),
    ])
    n, mean = PS.counter(db, "FETCH_SIZE", PS.KERNEL)
    assert n == 2 and mean == pytest.approx(200.0)


def test_trace_average_in_microseconds(tmp_path):
    db = _trace_db(tmp_path / "t.db", [
        (GEMM32, 1000, 6000), (GEMM64, 2000, 10000),   # 5 us and 8 us
        (GEMM_F32, 0, 10 ** 9), ("k_cg_step(SBatch, SGeo, SLay)", 0, 10 ** 9),
    ])
    n, avg = PS.trace_avg_us(db, PS.KERNEL)
    assert n == 2 and avg == pytest.approx(6.5)


def test_bench_scales_counters_by_the_copy_calibration(tmp_path, monkeypatch):
    import bench
    t = {"fetch_kib_per_dispatch": 500.0, "write_kib_per_dispatch": 300.0,
         "fetch_factor": 2.0, "write_factor": 1.0, "kernel_trace_avg_us": 6.5,
         "kernel_source_sha256_16": bench.kernel_source_hash()}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(t))
    monkeypatch.setattr(bench, "TRAFFIC", str(path))
    prof = bench.measured_profile()
    assert prof["traffic"] == pytest.approx(1024.0 * (500.0 * 2.0 + 300.0 * 1.0))
    assert prof["trace_avg_us"] == 6.5
    # counters taken on other kernel sources are not reported
    t["kernel_source_sha256_16"] = "0" * 16
    path.write_text(json.dumps(t))
    assert bench.measured_profile() is None



def test_cg_kernel_pattern_and_bench_sources(tmp_path):
    """The local-CG entry selects k_cg_coop only, and its source hash is the one
    bench.py checks before it reports the committed traffic."""
    import bench
    coop = "(anonymous namespace)::k_cg_coop((anonymous namespace)::SBatch, (anonymous namespace)::SGeo, " \
           "(anonymous namespace)::SLay, int, int, double*)"
    db = _trace_db(tmp_path / "t.db", [(coop, 0, 400000), (coop, 0, 200000), (GEMM32, 0, 10 ** 9)])
    pat, _, files = PS.KERNELS["cg_coop"]
    n, avg = PS.trace_avg_us(db, pat)
    assert n == 2 and avg == pytest.approx(300.0)
    assert PS.source_hash(files) == bench.kernel_source_hash()


def test_call_overlap_groups_calls_and_sums_concurrent_kernels(tmp_path):
    c = sqlite3.connect(tmp_path / "o.db")
    c.execute("create table kernels (name text, start integer, end integer, stream_id integer)")
    ms = 10 ** 6
    rows = [
        # call 0: two batches on streams 1 and 2, each 10 ms of kernels, overlapping
        ("void (anonymous namespace)::k_mpo_transpose(Batch, Geo, WsLayout)", 0, 1 * ms, 1),
        ("void (anonymous namespace)::k_zip_factor(Batch, Geo, WsLayout)", 1 * ms, 10 * ms, 1),
        ("void (anonymous namespace)::k_mpo_transpose(Batch, Geo, WsLayout)", 2 * ms, 3 * ms, 2),
        ("void (anonymous namespace)::k_zip_factor(Batch, Geo, WsLayout)", 3 * ms, 12 * ms, 2),
        ("__amd_rocclr_copyBuffer", 12 * ms, 13 * ms, 0),          # not a library kernel
        # call 1, 500 ms later: one batch
        ("void (anonymous namespace)::k_mpo_transpose(Batch, Geo, WsLayout)", 500 * ms, 501 * ms, 0),
        ("void (anonymous namespace)::k_rl_svd(Batch, Geo, WsLayout, int)", 501 * ms, 505 * ms, 0),
    ]
    c.executemany("insert into kernels values (?, ?, ?, ?)", rows)
    c.commit()
    c.close()
    out = PS.call_overlap(str(tmp_path / "o.db"), "k_mpo_transpose")
    assert len(out) == 2
    nb, nk, span, busy, st = out[0]
    assert (nb, nk, st) == (2, 4, [1, 2])
    assert span == pytest.approx(12.0) and busy == pytest.approx(20.0)
    nb, nk, span, busy, st = out[1]
    assert (nb, nk, st) == (1, 2, [0]) and span == pytest.approx(5.0) and busy == pytest.approx(5.0)

"""Host logic of the rocprofv3 summaries: the HBM bytes per dispatch of a
kernel family, on a stand-in counter database (the table and column names a
rocprofv3 run writes), so that no GPU or profiler is needed."""

import sqlite3

import pytest

from paper_1802_06952_amd import profiling as PR

KIB = 1024.0


def _db(path, rows):
    path.mkdir()
    con = sqlite3.connect(path / "run_results.db")
    con.execute("create table pmc_events (dispatch_id int, name text, counter_name text, "
                "counter_value real)")
    con.executemany("insert into pmc_events values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()


@pytest.fixture
def runs(tmp_path):
    # a plain copy of 1 MiB (the calibration: its fetch counter reads half the
    # bytes, its write counter all of them), then one dispatch of each kernel
    copy = "__amd_rocclr_copyBuffer(void*)"
    fetch = [(0, copy, "FETCH_SIZE", 512.0)]
    write = [(0, copy, "WRITE_SIZE", 1024.0)]
    kernels = [("void qs::k_wpass<4, 2>(qs::PassDesc const*)", 100.0, 400.0),
               ("void qs::k_xpass<4>(qs::XPassDesc const*)", 300.0, 600.0),
               ("void qs::k_zgemm_nt_f32<4, 2>(int, int)", 50.0, 10.0),
               ("void qs::k_zgemm_nt_f32d<4, 2>(int, int)", 70.0, 20.0)]
    for i, (n, f, w) in enumerate(kernels, start=1):
        fetch.append((i, n, "FETCH_SIZE", f))
        write.append((i, n, "WRITE_SIZE", w))
    _db(tmp_path / "fetch", fetch)
    _db(tmp_path / "write", write)
    return str(tmp_path / "fetch"), str(tmp_path / "write")


def test_calibrated_bytes_of_one_kernel(runs):
    d = PR.counter_summary(*runs, "k_wpass", 1 << 20)
    assert d["dispatches"] == 1
    assert d["calibration"]["fetch_factor"] == pytest.approx(0.5)
    assert d["calibration"]["write_factor"] == pytest.approx(1.0)
    # counters in KiB, divided by the copy's factors
    assert d["fetch_bytes_per_launch"] == pytest.approx(100.0 * KIB / 0.5)
    assert d["write_bytes_per_launch"] == pytest.approx(400.0 * KIB)
    assert d["hbm_bytes_per_launch"] == pytest.approx(200.0 * KIB + 400.0 * KIB)


def test_family_of_two_kernels_averages_their_dispatches(runs):
    d = PR.counter_summary(*runs, "k_wpass+k_xpass", 1 << 20)
    assert d["dispatches"] == 2
    assert d["fetch_bytes_per_launch"] == pytest.approx((100.0 + 300.0) / 2 * KIB / 0.5)
    assert d["write_bytes_per_launch"] == pytest.approx((400.0 + 600.0) / 2 * KIB)


def test_names_match_exactly_not_by_prefix(runs):
    plain = PR.counter_summary(*runs, "k_zgemm_nt_f32", 1 << 20)
    direct = PR.counter_summary(*runs, "k_zgemm_nt_f32d", 1 << 20)
    assert plain["dispatches"] == 1 and direct["dispatches"] == 1
    assert plain["write_bytes_per_launch"] == pytest.approx(10.0 * KIB)
    assert direct["write_bytes_per_launch"] == pytest.approx(20.0 * KIB)


def test_missing_kernel_is_an_error(runs):
    with pytest.raises(SystemExit):
        PR.counter_summary(*runs, "k_tail_ws", 1 << 20)

"""Host-side checks of the profile summariser (no GPU): kernel-name mapping
for every library kernel template, per-kernel source digests, and the
traffic scaling against the copy calibration on a synthetic counter CSV."""
import csv
import json
import os

import pytest

from paper_1805_05278_amd import rocprof_summary as rs


@pytest.mark.parametrize("symbol,name", [
    ("void miqr::k_chain_qr<256, true, 1>(miqr::ChainQRArgs)", "tsqr_chain_qr_leaf"),
    ("void miqr::k_chain_qr<128, true, 0>(miqr::ChainQRArgs)", "tsqr_chain_qr_leaf"),
    ("void miqr::k_chain_qr<256, true, 2>(miqr::ChainQRArgs)", "tsqr_chain_qr_leaf_rest"),
    ("void miqr::k_chain_qr_rest<256>(miqr::ChainQRArgs)", "tsqr_chain_qr_leaf_rest"),
    ("void miqr::k_chain_qr<256, false, 0>(miqr::ChainQRArgs)", "tsqr_chain_qr_tree"),
    ("void miqr::k_chain_down<2, 64, true, 8>(miqr::DownArgs)", "tsqr_down_leaf"),
    ("void miqr::k_chain_down<4, 128, true, 4>(miqr::DownArgs)", "tsqr_down_leaf"),
    ("void miqr::k_chain_down<4, 64, false, 4>(miqr::DownArgs)", "tsqr_down_tree"),
    ("miqr::k_tsqr_hr(miqr::HRArgs)", "tsqr_hr_root"),
    ("void miqr::k_gemm<128, 128, false, false, 0>(miqr::GemmArgs)", "gemm_f64"),
    ("void miqr::k_gemm<64, 64, true, false, 1>(miqr::GemmArgs)", "gemm_f32"),
    ("void miqr::k_gemm_bf16<128, 128, false, true>(miqr::GemmArgs)", "gemm_bf16"),
    ("miqr::k_splitk_reduce(double const*, int, long, long, double, double*, long, int)",
     "gemm_splitk_reduce"),
    ("void at::native::elementwise_kernel<128, 4, MulFunctor<double>>", "copy_calibration"),
    ("__amd_rocclr_copyBuffer", ""),
])
def test_kernel_names(symbol, name):
    assert rs.library_name(symbol) == name


def test_digest_per_kernel_sources():
    # A kernel's digest covers its own sources only: GEMM and TSQR records
    # are invalidated independently.
    g, t = rs.source_digest("gemm_f64"), rs.source_digest("tsqr_hr_root")
    assert g != t and len(g) == 16
    assert rs.source_digest("gemm_f32") == g
    assert rs.source_digest("tsqr_down_leaf") == t
    assert rs.source_digest("unknown") == rs.source_digest()


def _write_counters(path, rows):
    fields = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(fields, r)))


def test_traffic_scaled_by_copy(tmp_path):
    copy = "void at::native::elementwise_kernel<128, 4, MulFunctor<double>>"
    gemm = "void miqr::k_gemm<128, 128, false, false, 0>(miqr::GemmArgs)"
    kib = rs.COPY_BYTES / 1024.0
    fd, wd = tmp_path / "f", tmp_path / "w"
    fd.mkdir()
    wd.mkdir()
    # FETCH reads half of the copy's bytes, WRITE all of them: scales 2 and 1.
    _write_counters(fd / "x_counter_collection.csv",
                    [(copy, "FETCH_SIZE", kib / 2), (gemm, "FETCH_SIZE", 1000.0),
                     (gemm, "FETCH_SIZE", 3000.0)])
    _write_counters(wd / "x_counter_collection.csv",
                    [(copy, "WRITE_SIZE", kib), (gemm, "WRITE_SIZE", 500.0)])

    class A:
        fetch, write = str(fd), str(wd)
        command_fetch = command_write = "cmd"
        workload = "w1"
        out = str(tmp_path / "t.md")
        json = str(tmp_path / "t.json")

    rs.traffic(A)
    # A second workload's record is added beside the first.
    A.workload = "w2"
    rs.traffic(A)
    allrec = json.load(open(A.json))
    assert sorted(allrec) == ["w1", "w2"]
    rec = allrec["w1"]
    assert rec["_calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert rec["_calibration"]["write_scale"] == pytest.approx(1.0)
    g = rec["gemm_f64"]
    assert g["dispatches"] == 2
    assert g["hbm_bytes_per_launch"] == pytest.approx((2000.0 * 2.0 + 500.0) * 1024.0)
    assert g["source_digest"] == rs.source_digest("gemm_f64")
    assert os.path.exists(A.out)


def test_counters_table(tmp_path):
    blk = "void miqr::(anonymous namespace)::k_batched_blk<0, 5>(miqr::BatchHeader const*, int, int*, int*)"
    gemm = "void miqr::k_gemm<128, 128, false, false, 0>(miqr::GemmArgs)"
    d = tmp_path / "c"
    d.mkdir()
    _write_counters(d / "x_counter_collection.csv",
                    [(gemm, "MfmaUtil", 60.0), (gemm, "MfmaUtil", 40.0), (blk, "MfmaUtil", 10.0),
                     (gemm, "VALUBusy", 5.0), (blk, "VALUBusy", 30.0)])

    class A:
        dir = str(d)
        command = "cmd"
        workload = "w"
        out = str(tmp_path / "c.md")

    rs.counters(A)
    text = open(A.out).read()
    assert "| gemm_f64 | 2 | 50 | 5 |" in text
    assert "| batched_blk_f64 | 1 | 10 | 30 |" in text

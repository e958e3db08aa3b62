"""Host logic of bench.py's counter-based traffic (no GPU): a traffic record
made from FETCH_SIZE / WRITE_SIZE counter files, the calibration factors
from the copy kernel, and the rules that turn it into bytes per launch or
into null (another source of the kernel, another k-set for the structure
factors)."""
import csv
import json
import os

import pytest

import bench


def _counter_dir(tmp_path, name, counter, values):
    d = tmp_path / name
    d.mkdir()
    with open(d / "run_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for kernel, vals in values.items():
            for v in vals:
                w.writerow({"Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": v})
    return str(d)


COPY = "void at::native::vectorized_elementwise_kernel<4, MulFunctor>(int)"
SPLIT = "void cpm::(anonymous namespace)::block_matvec_split_kernel<float, 2>(float const*)"
SF = "cpm::(anonymous namespace)::sf_gemm_kernel(double const*, double const*)"


@pytest.fixture()
def record(tmp_path):
    kib = bench.CALIB_BYTES / 1024.0
    fetch = _counter_dir(tmp_path, "fetch", "FETCH_SIZE",
                         {COPY: [kib / 2] * 3, SPLIT: [100.0, 90.0, 0.5], SF: [40.0, 40.0]})
    write = _counter_dir(tmp_path, "write", "WRITE_SIZE",
                         {COPY: [kib] * 3, SPLIT: [10.0, 12.0, 0.0], SF: [8.0, 8.0]})
    with open(str(tmp_path / "fetch") + ".json", "w") as fh:
        fh.write(json.dumps({"config": {"n_kvec": 1181, "kmax_override": 0.3}}) + "\n")
    out = str(tmp_path / "traffic.json")
    bench.summarize_pmc(fetch, write, out)
    with open(out) as fh:
        return out, json.load(fh)


def test_record_contents(record):
    _, rec = record
    cal = rec["calibration"]
    assert cal["fetch_factor"] == pytest.approx(2.0) and cal["write_factor"] == pytest.approx(1.0)
    k = rec["kernels"]
    # medians over the dispatches (gated no-op launches do not pull them down)
    assert k["block_matvec_split_kernel<float, 2>"] == {"dispatches": 3, "fetch_kib": 90.0,
                                                        "write_kib": 10.0}
    assert k["sf_gemm_kernel"]["fetch_kib"] == 40.0
    assert rec["run_config"] == {"n_kvec": 1181, "kmax_override": 0.3}
    for f in ("cg.hip", "rhs.hip"):
        assert rec["source_sha256"][f] == bench._sha256(os.path.join(bench.CSRC, f))


def test_bytes_per_launch(record):
    path, _ = record
    # FETCH_SIZE x 2 + WRITE_SIZE x 1, KiB -> bytes
    assert bench.traffic_bytes(path, "matvec_f32", 2) == pytest.approx(1024.0 * (90.0 * 2 + 10.0))
    assert bench.traffic_bytes(path, "sf", 2, n_kvec=1181) == pytest.approx(1024.0 * (80.0 + 8.0))


def test_null_when_stale(record, tmp_path):
    path, rec = record
    # the structure factors of another k-set
    assert bench.traffic_bytes(path, "sf", 2, n_kvec=482337) is None
    # a kernel the record does not hold
    assert bench.traffic_bytes(path, "matvec_f64", 2) is None
    # the source of the block product changed since the counters were taken
    rec["source_sha256"]["cg.hip"] = "0" * 64
    stale = str(tmp_path / "stale.json")
    with open(stale, "w") as fh:
        json.dump(rec, fh)
    assert bench.traffic_bytes(stale, "matvec_f32", 2) is None
    assert bench.traffic_bytes(stale, "sf", 2, n_kvec=1181) is not None
    assert bench.traffic_bytes(str(tmp_path / "missing.json"), "matvec_f32", 2) is None

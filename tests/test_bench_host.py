"""Host logic of the benchmark (no GPU): the algorithmic bytes of a
stream-collide launch, the scaling of rocprofv3 byte counters by a plain
copy of known size, and the use of a stored traffic record only on the
workload, storage precision and kernel sources it was taken on."""
import csv
import json

import numpy as np

import bench


def test_algorithmic_bytes_per_launch():
    flags = np.zeros((4, 4, 4), np.uint8)
    flags[1, 1, 1:3] = 1  # two liquid cells
    flags[2, 2, 2] = 2    # one interface cell
    flags[0, 0, 0] = 3
    for prec, s, r in (("f32", 4, 4), ("f16", 2, 4), ("bf16", 2, 4), ("f64", 8, 8)):
        bl, bi, nl, ni, nbox = bench.sc_bytes(flags, prec)
        assert (nl, ni) == (2, 1)
        # the fluid bounding box: z 1..2, y 1..2, x 1..2
        assert nbox == 8
        # 19 reads and 19 writes of a distribution per liquid cell, 1 flag byte per fluid-box cell
        assert bl == 2 * 38 * s + 8
        # the same per interface cell, plus m (read, write), rho, K, phi and a status byte
        assert bi == 38 * s + 5 * r + 1


def _csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for kernel, value in rows:
            w.writerow({"Kernel_Name": kernel, "Counter_Name": "X", "Counter_Value": value})


def test_counter_scaling_by_a_plain_copy(tmp_path):
    f, w, cf, cw = (str(tmp_path / n) for n in ("f.csv", "w.csv", "cf.csv", "cw.csv"))
    sc = "void fslbm::k_stream_collide<fslbm::Prec<1>, 0, 0>(fslbm::Batch<fslbm::Prec<1> >)"
    _csv(f, [(sc, 1000.0), (sc, 3000.0), ("void fslbm::k_curv_lsqr4<fslbm::Prec<1> >", 99.0)])
    _csv(w, [(sc, 500.0)])
    # a copy of 2^28 floats (1 GiB each way) whose counters read half the
    # bytes fetched and all the bytes written
    _csv(cf, [("void at::native::vectorized_elementwise_kernel<AUnaryFunctor>", (1 << 30) / 2048.0)])
    _csv(cw, [("void at::native::vectorized_elementwise_kernel<AUnaryFunctor>", (1 << 30) / 1024.0)])
    rec = bench.traffic_from_counters(f, w, cf, cw, workload_note="droplet-sweep", precision="f32")
    assert rec["dispatches"] == [2, 1]
    assert abs(rec["fetch_scale"] - 2.0) < 1e-12 and abs(rec["write_scale"] - 1.0) < 1e-12
    assert rec["bytes_per_launch"] == int(1024 * (2000.0 * 2.0 + 500.0))
    assert (rec["workload"], rec["precision"]) == ("droplet-sweep", "f32")


def test_stored_traffic_only_where_it_was_taken(tmp_path, monkeypatch):
    rec = {"source_sha256": bench.stream_source_hash(), "workload": "droplet-sweep", "precision": "f32",
           "bytes_per_launch": 1}
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.stored_traffic("droplet-sweep", "f32") == rec
    assert bench.stored_traffic("ellipsoid", "f32") is None
    assert bench.stored_traffic("droplet-sweep", "f16") is None
    rec["source_sha256"] = "0" * 64
    path.write_text(json.dumps(rec))
    assert bench.stored_traffic("droplet-sweep", "f32") is None


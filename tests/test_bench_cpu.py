"""Host logic of bench.py: the committed counter record is used only for the
kernels it was taken on."""
import json

import numpy as np

import bench

V = "hydroagg gfx950 src aaaaaaaaaaaa kernels 111111111111"
K = "void hydro::hydro_lds8_kernel<11, 14>(hydro::DevDesc const*, int, double, double, double*)"


def write(tmp_path, version, workload="4096x8^3 F=11", kernel=K):
    p = tmp_path / "rec.json"
    p.write_text(json.dumps({"kernel_version": version, "kernel": kernel, "workload": workload,
                             "traffic_bytes_per_launch": 1129123938.3}))
    return str(p)


def test_kernels_hash_parsing():
    assert bench.kernels_hash(V) == "111111111111"
    assert bench.kernels_hash("hydroagg gfx950 src aaaaaaaaaaaa") is None
    assert bench.kernels_hash("") is None
    assert bench.kernels_hash("x kernels") is None


def test_record_follows_the_kernels_not_the_host_code(tmp_path):
    p = write(tmp_path, V)
    other_host = "hydroagg gfx950 src bbbbbbbbbbbb kernels 111111111111"
    assert bench.measured_traffic(other_host, "4096x8^3 F=11", "hydro_lds8_kernel<11,14>", p) == 1129123938
    other_kernels = "hydroagg gfx950 src aaaaaaaaaaaa kernels 222222222222"
    assert bench.measured_traffic(other_kernels, "4096x8^3 F=11", "hydro_lds8_kernel<11,14>", p) is None


def test_record_needs_same_workload_and_kernel(tmp_path):
    p = write(tmp_path, V)
    assert bench.measured_traffic(V, "2048x8^3 F=11", "hydro_lds8_kernel<11,14>", p) is None
    assert bench.measured_traffic(V, "4096x8^3 F=11", "hydro_q4_kernel<11,14>", p) is None


def test_old_records_without_a_kernels_hash_are_not_used(tmp_path):
    p = write(tmp_path, "hydroagg gfx950 src aaaaaaaaaaaa")
    assert bench.measured_traffic(V, "4096x8^3 F=11", "hydro_lds8_kernel<11,14>", p) is None
    missing = str(tmp_path / "missing.json")
    assert bench.measured_traffic(V, "4096x8^3 F=11", "hydro_lds8_kernel<11,14>", missing) is None


def test_fp64_rate_from_the_record(tmp_path):
    p = tmp_path / "fp64.json"
    p.write_text(json.dumps({"kernel_version": V, "kernel": K, "workload": "4096x8^3 F=11",
                             "fp64_flop_per_launch": 3.0e9, "valu_insts_per_wave": 5000.0}))
    r = bench.measured_fp64(V, "4096x8^3 F=11", "hydro_lds8_kernel<11,14>", 0.3, str(p))
    assert r["flop_per_launch"] == 3000000000 and r["achieved_tflops"] == 10.0
    assert r["frac"] == round(10.0 / 78.6, 4)
    other = "hydroagg gfx950 src aaaaaaaaaaaa kernels 999999999999"
    assert bench.measured_fp64(other, "4096x8^3 F=11", "hydro_lds8_kernel<11,14>", 0.3, str(p)) is None


def test_per_subgrid_metric_sees_what_the_pooled_one_cannot():
    from tests.gpu_util import normwise, normwise_each
    rng = np.random.default_rng(0)
    ref = rng.uniform(0.5, 1.5, size=(3, 2, 4, 4, 4))
    ref[1] *= 1e-10                      # a sub-grid of tiny values (atmosphere)
    got = ref.copy()
    got[1, 0, 2, 2, 2] *= 1 + 1e-6       # an error of 1e-6 relative inside it
    assert normwise(got, ref).max() < 1e-12
    each = normwise_each(got, ref)
    assert each.shape == (3, 2)
    assert abs(each[1, 0] - 1e-6 * ref[1, 0, 2, 2, 2] / np.abs(ref[1, 0]).max()) < 1e-12
    assert each[0].max() == 0 and each[2].max() == 0 and each[1, 1] == 0
    zero = np.zeros_like(ref)
    assert normwise_each(zero, zero).max() == 0
    assert normwise_each(zero + 1e-300, zero)[0, 0] == 1e-300

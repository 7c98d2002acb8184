"""Host-side logic that needs no GPU: the autotuner's candidate space and shape key,
the rocprofv3 summary reader, and the benchmark's one-GPU guard."""
import json
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_autotune_candidates_and_shape_key():
    torch = pytest.importorskip("torch")  # noqa: F841  (autotune imports the binding)
    from paper_2302_11719_amd import autotune

    c = autotune.candidates(256)
    assert c[0] == dict(pipeline=1, block=0, tile=0, grid=0)
    assert len(c) == 1 + (4 * 3 - 1) * 4  # block 512 has no 4-sample tiles
    for d in c[1:]:
        assert d["tile"] % d["block"] == 0 and d["tile"] <= 1024 and d["grid"] in (0, 256, 512, 1024)
    fake = types.SimpleNamespace(K=[100, 300], T=[20, 40], B=2, track=types.SimpleNamespace(obs_max=0))
    k1 = autotune.shape_key(fake, 256)
    assert k1 == autotune.shape_key(fake, 256) and k1 != autotune.shape_key(fake, 128)
    fake2 = types.SimpleNamespace(K=[100, 301], T=[20, 40], B=2, track=types.SimpleNamespace(obs_max=64))
    assert autotune.shape_key(fake2, 256) != k1
    # sum K = 400: round(8 log2 400) = 69
    assert k1 == "B2-sk69-kmax300-tmax40-tmean30.0-obs0-cu256"


def test_autotune_key_rejects_bad_arguments():
    """smppi_autotune_key validates its host arguments (no device needed)."""
    pytest.importorskip("torch")
    import ctypes

    import numpy as np

    from paper_2302_11719_amd import _lib as L

    k = np.array([0, 10], dtype=np.int64)
    t = np.array([0, 5], dtype=np.int32)
    pk, pt = k.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), t.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    buf = ctypes.create_string_buffer(64)
    assert L.lib().smppi_autotune_key(1, pk, pt, 0, 8, buf, 64) == 0
    assert buf.value == b"B1-sk27-kmax10-tmax5-tmean5.0-obs0-cu8"
    assert L.lib().smppi_autotune_key(0, pk, pt, 0, 8, buf, 64) == 1
    assert L.lib().smppi_autotune_key(1, None, pt, 0, 8, buf, 64) == 1
    assert L.lib().smppi_autotune_key(1, pk, pt, 0, 8, buf, 10) == 1  # key does not fit
    assert L.lib().smppi_autotune_candidates(8, None, 0) == 45


def test_profile_summary_reads_counters_and_scales_traffic(tmp_path):
    from paper_2302_11719_amd import profile_summary as ps

    def write(d, rows):
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, "p_counter_collection.csv"), "w") as fh:
            fh.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
            for r in rows:
                fh.write(",".join(str(x) for x in r) + "\n")

    n = 1 << 20
    write(tmp_path / "f", [(1, '"__amd_rocclr_copyBuffer"', '"FETCH_SIZE"', n / 2048),
                           (2, '"void (anonymous namespace)::k_fused<0, 256, 1, true>(FusedArgs)"', '"FETCH_SIZE"', 10.0),
                           (3, '"void (anonymous namespace)::k_fused<0, 256, 1, true>(FusedArgs)"', '"FETCH_SIZE"', 30.0)])
    write(tmp_path / "w", [(1, '"__amd_rocclr_copyBuffer"', '"WRITE_SIZE"', n / 1024),
                           (2, '"void (anonymous namespace)::k_fused<0, 256, 1, true>(FusedArgs)"', '"WRITE_SIZE"', 4.0)])
    s = ps.traffic_summary(str(tmp_path / "f"), str(tmp_path / "w"), "k_fused", n)
    k = s["kernels"]["k_fused<0, 256, 1, true>"]
    assert s["fetch_factor"] == pytest.approx(2.0) and s["write_factor"] == pytest.approx(1.0)
    assert k["fetch_bytes"] == pytest.approx(20.0 * 1024 * 2.0) and k["write_bytes"] == pytest.approx(4096.0)
    out = tmp_path / "t.md"
    ps.write_md(str(out), "t", "cmd", "", s)
    b, p = ps.load_traffic(str(out), "k_fused")
    assert b == pytest.approx(k["traffic_bytes"]) and p["digest"] == ps.kernel_sources_digest()
    p["digest"] = "0" * 16
    ps.write_md(str(out), "t", "cmd", "", p)
    assert ps.load_traffic(str(out), "k_fused")[0] is None


def test_profile_summary_reads_bytes_by_request_size(tmp_path):
    """With the request-size counters the read bytes are 32/64/128 per request,
    unscaled; the copy kernel only yields a check factor."""
    from paper_2302_11719_amd import profile_summary as ps

    def write(d, rows):
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, "p_counter_collection.csv"), "w") as fh:
            fh.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
            for r in rows:
                fh.write(",".join(str(x) for x in r) + "\n")

    n = 1 << 20
    kf = '"void (anonymous namespace)::k_fused<0, 256, 1, true>(FusedArgs)"'
    rows = [(1, '"__amd_rocclr_copyBuffer"', '"TCC_EA0_RDREQ_32B_sum"', 0),
            (1, '"__amd_rocclr_copyBuffer"', '"TCC_EA0_RDREQ_64B_sum"', 0),
            (1, '"__amd_rocclr_copyBuffer"', '"TCC_EA0_RDREQ_128B_sum"', n // 128)]
    for disp, (a, b, c) in ((2, (1, 10, 2)), (3, (3, 30, 6))):
        rows += [(disp, kf, '"TCC_EA0_RDREQ_32B_sum"', a), (disp, kf, '"TCC_EA0_RDREQ_64B_sum"', b),
                 (disp, kf, '"TCC_EA0_RDREQ_128B_sum"', c)]
    write(tmp_path / "f", rows)
    write(tmp_path / "w", [(1, '"__amd_rocclr_copyBuffer"', '"WRITE_SIZE"', n / 1024), (2, kf, '"WRITE_SIZE"', 1.0)])
    s = ps.traffic_summary(str(tmp_path / "f"), str(tmp_path / "w"), "k_fused", n)
    k = s["kernels"]["k_fused<0, 256, 1, true>"]
    assert s["read_method"] == "request sizes" and s["fetch_factor"] == pytest.approx(1.0)
    mean_read = ((32 + 640 + 256) + (96 + 1920 + 768)) / 2
    assert k["fetch_bytes"] == pytest.approx(mean_read)
    assert k["traffic_bytes"] == pytest.approx(mean_read + 1024.0)


def test_derived_counter_rates():
    """FLOP from the instruction mix (64 lanes, FMA = 2), rates against the peaks, and
    VALU issue utilisation from GRBM cycles summed over the XCDs."""
    from paper_2302_11719_amd import profile_summary as ps
    cs = {"SQ_INSTS_VALU_FLOPS_FP32": 1.0e6, "duration_ns": 1.0e4, "GRBM_GUI_ACTIVE": 8 * 2.0e4,
          "SQ_INSTS_VALU": 2.56e6, "SQ_ACTIVE_INST_VALU": 5.12e6}
    d = ps.derived(cs, simds=1024, xcds=8)
    assert d["fp32_flop_per_dispatch"] == pytest.approx(6.4e7)
    assert d["fp32_tflops"] == pytest.approx(6.4e7 / 1e-5 / 1e12)
    assert d["frac_fp32_peak_packed"] == pytest.approx(6.4e12 / 157.3e12)
    assert d["frac_fp32_peak_unpacked"] == pytest.approx(2 * 6.4e12 / 157.3e12)
    assert d["gui_active_ghz"] == pytest.approx(2.0)
    assert d["valu_issue_util"] == pytest.approx(4 * 2.56e6 / (1024 * 2.0e4))
    assert d["active_inst_valu_util"] == pytest.approx(1.0)
    assert ps.derived({"duration_ns": 1.0}) == {}


def test_short_kernel_names():
    from paper_2302_11719_amd.profile_summary import short_name

    assert short_name("void (anonymous namespace)::k_fused<0, 192, 1, true>((anonymous namespace)::FusedArgs)") \
        == "k_fused<0, 192, 1, true>"
    assert short_name("void smppi::k_repair<float, 0>(smppi::RepairArgs<float>)") == "k_repair<float, 0>"
    assert short_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]

"""CPU checks of the C ABI: the library loads, exports every function the header
declares, and the ctypes struct layouts equal the C layouts (checked with a
C program compiled against include/smppi.h).  No compute calls: no GPU here."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2302_11719_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smppi.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smppi_[a-z_]+)\s*\(", text)))


def test_header_declares_the_five_calls():
    names = _declared_functions()
    for n in ("smppi_rollout", "smppi_weights", "smppi_update", "smppi_rollout_backward", "smppi_shield_repair"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    names = _declared_functions()
    assert set(names) == set(L.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (smppi_\w+)", out))
    assert set(names) <= exported


def test_abi_version_and_status_strings():
    lib = L.lib()
    hdr = open(os.path.join(ROOT, "include", "smppi.h")).read()
    ver = int(re.search(r"#define SMPPI_ABI_VERSION (\d+)", hdr).group(1))
    assert lib.smppi_abi_version() == ver == L.ABI_VERSION
    assert lib.smppi_status_string(0) == b"ok"
    assert lib.smppi_status_string(4) == b"no device"


def test_null_arguments_are_rejected_before_any_launch():
    lib = L.lib()
    assert lib.smppi_create(0, None) == 1
    assert lib.smppi_rollout(None, None, None, None, None, None, None, None, None, None, None, None) == 1
    assert lib.smppi_plan_launch(None, None) == 1


def test_create_without_gpu_reports_no_device():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    assert L.lib().smppi_create(0, ctypes.byref(h)) == L.ERR_NO_DEVICE
    assert not h.value


def test_struct_layouts_match_c(tmp_path):
    structs = {"smppi_model": L.Model, "smppi_cost": L.Cost, "smppi_noise": L.Noise, "smppi_batch": L.Batch,
               "smppi_track": L.Track, "smppi_objective": L.Objective, "smppi_repair_opts": L.RepairOpts,
               "smppi_plan_opts": L.PlanOpts, "smppi_plan_buffers": L.PlanBuffers,
               "smppi_curv_track": L.CurvTrack, "smppi_wheels": L.Wheels}
    fields = {"smppi_batch": ["k_off", "t_off", "dtype"], "smppi_track": ["window", "obs_max", "obs"],
              "smppi_cost": ["gamma", "sigma"], "smppi_plan_opts": ["repair_opts", "dist", "use_graph", "n_dist", "pipeline", "fuse_shield"],
              "smppi_repair_opts": ["step", "objective", "method", "memory"], "smppi_model": ["u_hi"],
              "smppi_curv_track": ["ds", "half_width", "n_max"], "smppi_wheels": ["I_w", "C_x"]}
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "smppi.h"', "int main(void){"]
    for cname in structs:
        src.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f in fields.get(cname, []):
            src.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for f in fields.get(cname, []):
            pyf = "lambda_" if f == "lambda" else f
            assert int(got[f"{cname}.{f}"]) == getattr(py, pyf).offset, f"{cname}.{f}"


def test_hot_calls_never_allocate():
    """Device memory is allocated only by smppi_create, smppi_reserve_batch and the plan
    calls: the scratch-growing helpers are called from smppi_reserve_batch alone, and the
    hot calls check the reserved size instead (SMPPI_ERR_SHAPE)."""
    src = open(os.path.join(ROOT, "paper_2302_11719_amd", "csrc", "smppi.hip")).read()
    body = lambda name: src[src.index(name):]
    for helper in ("ensure_scratch(", "ensure_tickets("):
        callers = [m.start() for m in re.finditer(re.escape(helper), src)]
        # the definition, and one call inside smppi_reserve_batch
        defs = [i for i in callers if src[max(0, i - 8):i].endswith("smppi::")]
        calls = [i for i in callers if i not in defs]
        start = src.index('smppi_reserve_batch(smppi_ctx ctx')
        end = src.index("\n}\n", start)
        assert len(defs) == 1 and calls and all(start < i < end for i in calls), helper
    assert "hipMalloc" not in body("// ------------------------------------------------------------------ rollout")
    hdr = open(HEADER).read()
    assert "No call that enqueues work allocates" in hdr and "smppi_reserve_batch" in hdr

"""Host-side checks of the C-ABI library (no GPU): it loads, it exports every
entry point include/cfust.h declares, and the binding refuses to run without
it.  Also checks host logic that needs no device: the lattice design inputs
and the integral bookkeeping of the bench."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cfust.h")
LIB = os.path.join(ROOT, "paper_1606_02054_amd", "libcfust.so")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:cfust_status|const char \*)\s*(\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_1606_02054_amd import build
        build.build()
    return LIB


def test_header_declares_the_four_calls():
    names = declared_functions()
    for f in ("cfust_estep", "cfust_mstep", "cfust_loglik", "mvt_cdf_batch"):
        assert f in names


def test_library_exports_every_declared_symbol(built):
    lib = ctypes.CDLL(built)
    for name in declared_functions():
        assert hasattr(lib, name), name
    from paper_1606_02054_amd import _binding
    assert sorted(_binding.EXPORTS) == declared_functions()


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1606_02054_amd import _binding
    with pytest.raises(RuntimeError, match="not found"):
        _binding._lib = None
        _binding.load(str(tmp_path / "missing.so"))
    _binding._lib = None


def test_status_codes_match_header():
    text = open(HEADER).read()
    from paper_1606_02054_amd import _binding
    for code, name in _binding.STATUS.items():
        assert re.search(rf"{name}\s*=\s*{code}\b", text), name
    for bit, name in _binding.DEV_BITS.items():
        m = re.search(rf"CFUST_DEV_{name}\s*\(1 << (\d+)\)", text)
        assert m and (1 << int(m.group(1))) == bit, name


def test_lattice_design_inputs():
    from cfust_inputs import make_design
    d = make_design(4096, 8, seed=3)
    assert d.z.shape == (8,) and d.z.dtype == np.int32
    assert d.z[0] == 1 and np.all(d.z % 2 == 1) and np.all(d.z < 4096)
    assert d.shifts.shape == (8, 8) and np.all((d.shifts >= 0) & (d.shifts < 1))
    assert np.array_equal(make_design(4096, 8, seed=3).shifts, d.shifts)


def test_bench_flop_bookkeeping():
    import bench
    assert bench.integral_dims(4) == [4, 4, 3, 3, 3, 3, 2, 2, 2, 2, 2, 2]
    assert bench.integral_dims(2) == [2, 2]
    assert len(bench.integral_dims(8)) == 38
    # the counter-measured flops per lattice point are used only for the kernel
    # sources they were measured on
    if bench.counters_current():
        assert all(bench.lattice_flops_per_point(m) > 0 for m in range(2, 9))
    else:
        assert bench.lattice_flops_per_point(2) is None


def test_bench_counter_summary(tmp_path):
    """The counter summary of the bench reads rocprofv3's pmc_events table:
    per dimension m, FP32 flops per lattice point = (2 FMA + MUL + ADD +
    TRANS) x 64 lanes / (waves x points per wave), VALU issue per CU and cycle from
    GRBM_GUI_ACTIVE summed over the 8 XCDs, and the dual-issued share."""
    import sqlite3
    import bench
    db = tmp_path / "x.db"
    con = sqlite3.connect(db)
    con.execute("create table pmc_events (dispatch_id int, name text, duration real, counter_name text, "
                "counter_value real)")
    vals = {"SQ_WAVES": 10.0, "SQ_INSTS_VALU_FMA_F32": 300.0, "SQ_INSTS_VALU_MUL_F32": 50.0,
            "SQ_INSTS_VALU_ADD_F32": 20.0, "SQ_INSTS_VALU_TRANS_F32": 10.0, "SQ_INSTS_VALU": 512.0,
            "SQ_ACTIVE_INST_VALU2": 128.0, "GRBM_GUI_ACTIVE": 8.0}
    for k, v in vals.items():
        con.execute("insert into pmc_events values (1, 'void cfust::k_estep_qmc<3, true, 1, true>(x)', 1.0, ?, ?)",
                    (k, v))
    con.execute("insert into pmc_events values (2, 'void cfust::k_mstep_reduce(x)', 1.0, 'SQ_WAVES', 5.0)")
    con.commit()
    con.close()
    r = bench.summarize_counters([str(db)], points_per_wave=4)
    assert list(r) == [3]
    assert r[3]["flops_per_point"] == (600 + 50 + 20 + 10) * 64 / 40.0
    assert r[3]["valu_per_cu_cycle"] == 512.0 / 256.0 / 1.0
    assert r[3]["dual_issue_frac"] == 0.5


def test_bench_refuses_several_gpus():
    """The bench measures one GPU; --gpus above 1 exits with status 2 and a
    JSON line saying so, before any GPU work."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert msg["n_gpus"] == 2 and "one GPU" in msg["error"]

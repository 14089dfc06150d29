"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
byte counts behind the roofline figure, and the element block the CPU
baseline runs on."""
import os
import subprocess
import sys

import numpy as np
import pytest

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, REPO)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(REPO, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_model2_bytes_per_node():
    """3D FP64: lift reads U (5 words) and writes tau and grad c (9); rhs reads
    U, G and dU and writes U and dU (232 B, 192 B in the first stage, whose
    A coefficient is zero); with G in FP32 the G words take 4 bytes."""
    assert bench.bytes_per_node(3, False, False) == {"lift": 112, "rhs": 232}
    assert bench.bytes_per_node(3, True, False) == {"lift": 112, "rhs": 192}
    assert bench.bytes_per_node(3, False, True) == {"lift": 76, "rhs": 196}
    # 2D: 4 state words, 3 tau + 2 grad c
    assert bench.bytes_per_node(2, False, False) == {"lift": 72, "rhs": 168}


def test_nsk_bytes_per_node():
    """3D original NSK path: 4 state words, 6 tau and 3 grad rho: lift 104 B,
    second lifting 128 B (reads grad rho, tau, rho; writes Sigma), rhs 176 B
    (144 B in the first stage): 408 B per node and stage."""
    b = bench.nsk_bytes_per_node(3, False)
    assert b == {"lift": 104, "lap": 128, "rhs": 176}
    assert sum(b.values()) == 408
    assert bench.nsk_bytes_per_node(3, True)["rhs"] == 144


def test_sample_block_picks_the_sub_box():
    nel = (6, 5, 4)
    E = 6 * 5 * 4
    U = np.arange(2 * E * 3, dtype=float).reshape(2, E, 3)
    block = [(1, 3), (2, 2), (0, 2)]
    got = bench.sample_block(U, nel, block)
    assert got.shape == (2, 3 * 2 * 2, 3)
    # x fastest, then y, then z, as in the full state
    want = [x + 6 * (y + 5 * z) for z in (0, 1) for y in (2, 3) for x in (1, 2, 3)]
    assert np.array_equal(got, U[:, want, :])
    nel2 = (4, 3)
    U2 = np.arange(12 * 2, dtype=float).reshape(1, 12, 2)
    got2 = bench.sample_block(U2, nel2, [(2, 2), (1, 2)])
    assert np.array_equal(got2, U2[:, [2 + 4 * 1, 3 + 4 * 1, 2 + 4 * 2, 3 + 4 * 2], :])


def test_counter_record_only_for_its_own_shape():
    """The committed counter record is reported only for its workload,
    precision and launch shape."""
    assert bench.counter_traffic("2d-droplets", "fp64", (0, 3)) is None
    assert bench.counter_traffic("3d-collision", "fp64", (1, 5)) is None
    assert bench.counter_traffic("3d-collision", "mixed", (1, 5)) is None
    # each precision gets its own record, where one exists
    f, m = (bench.counter_traffic("3d-collision", p, (0, 3)) for p in ("fp64", "mixed"))
    if f is not None and m is not None:
        assert f["source"] != m["source"] and "fp64" in f["source"] and "mixed" in m["source"]


def test_dof_stage_rate_units():
    """256 nodes, five stages per step, 34.5 microseconds per step: 3.71e7
    DOF-stage updates per second (the 1D slab workload's figures)."""
    assert bench.dof_stage_rate(256, 1, 34.5e-6) == pytest.approx(256 * 5 / 34.5e-6, rel=1e-12)
    assert bench.dof_stage_rate(256, 1, 34.5e-6) == pytest.approx(3.71e7, rel=1e-3)
    assert bench.dof_stage_rate(230400, 200, 0.0352) == pytest.approx(6.545e9, rel=1e-3)

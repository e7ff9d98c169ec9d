"""bench.py's host-side pieces that need no GPU: the refusal of more than
one GPU and of zero repetition counts, and the issue fractions read from a rocprofv3 SQ summary (the
committed one and a hand-made one with known figures)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert "exactly one GPU" in out.stdout


@pytest.mark.parametrize("flag", ["--plain-steps", "--kernel-reps", "--roundtrip-reps"])
def test_zero_repetitions_are_refused(flag):
    # argparse rejects the value before anything is imported or timed
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), flag, "0"],
                         capture_output=True, text=True, timeout=120)
    assert out.returncode == 2
    assert f"{flag} must be at least 1" in out.stderr


def test_issue_fractions_hand_made(tmp_path):
    p = tmp_path / "sq.txt"
    p.write_text(
        "# header\n\n"
        "kernel counter dispatches mean min max\n"
        "void mpld::reg_batched_kernel<false, 3, false>(x   SQ_INSTS_SALU   2   614400.0  1 2\n"
        "void mpld::reg_batched_kernel<false, 3, false>(x   SQ_INSTS_VALU   2   307200.0  1 2\n"
        "void mpld::reg_batched_kernel<false, 3, false>(x        SQ_WAVES   2     3472.0  1 2\n"
        "__amd_rocclr_copyBuffer                            SQ_INSTS_SALU   4      999.0  1 2\n")
    # 1 us at 2.4 GHz on 256 CUs is 614,400 CU-cycles
    got = bench.issue_fractions(str(p), 1e-3)
    assert got["salu_frac"] == pytest.approx(1.0)
    assert got["valu_frac"] == pytest.approx(0.5)
    assert got["waves"] == 3472.0
    assert bench.issue_fractions(str(tmp_path / "missing.txt"), 1e-3) is None


def test_issue_fractions_committed_summary():
    p = os.path.join(ROOT, "profiles", "reg_batched_kernel_200k-k3-d80_pmc_sq.txt")
    got = bench.issue_fractions(p, 4.4e-3)
    assert got is not None
    assert 0.0 < got["salu_frac"] < 1.0 and 0.0 < got["valu_frac"] < 1.0


def test_cpu_legs_agree_with_the_batch_and_flag_a_mismatch():
    """The CPU legs reproduce the per-component status and node counts they
    are given (here the oracle's own decomposition of the small workload) and
    report agree = False when one node count differs."""
    import numpy as np

    import oracle
    import workload
    from workload.configs import CONFIGS
    w = CONFIGS[0]
    rects, _ = workload.generate(w.n_rects, w.side_nm, w.seed)
    ref = oracle.decompose(oracle.build_graph(rects, w.dmin_nm, w.split_len_nm), w.k, w.budget)
    comps = ref.comps
    one, alln = bench.cpu_legs(rects, w, 0.05, comps)
    assert one["agree"] and alln["agree"]
    assert one["cores"] == 1 and alln["cores"] >= 1
    assert one["value"] > 0 and alln["value"] > 0
    bad = comps.copy()
    bad["nodes"][0] += 1
    one, _ = bench.cpu_legs(rects, w, 0.05, bad)
    assert not one["agree"]
    assert np.array_equal(comps["nodes"], ref.comps["nodes"])

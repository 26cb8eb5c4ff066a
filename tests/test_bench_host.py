"""Host-side logic of bench.py: the per-pass byte model, the profile lookups
that feed the roofline's traffic and VALU figures, and the one-GPU rule.
No device work."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

psn = pytest.importorskip("paper_1612_01799_amd")


@pytest.mark.parametrize("dt", ["f32", "f64", "split"])
@pytest.mark.parametrize("n", [48, 160, 512])
def test_pass_bytes_add_up_to_the_library_figure(n, dt):
    """The five passes' algorithmic bytes (each array read and written once)
    sum to the plan's algorithmic bytes per solve."""
    info = psn.Plan(n, 4.0, 1e-12, dt).info()
    assert sum(bench.pass_bytes(n, dt)) == pytest.approx(info["algorithmic_bytes"], rel=1e-12)


def _summary(path, digest, value):
    path.write_text(
        "# a profile summary\n"
        f"# kernel sources sha256[:16] (psn_device.h + psn_passes.h): {digest}\n"
        "kernel                               disp  read_GB write_GB total_GB\n"
        "psn::p3p_conv<512, 1, 8, 32, 1, 2>     15    2.687    2.147    " + f"{value:.3f}\n"
        "psn::p4p_inv<512, 1, 8, 64, false>     15    2.148    1.074    3.221\n")


def test_profile_value_reads_the_row_by_column(tmp_path):
    p = tmp_path / "s.txt"
    _summary(p, bench._sources_digest(), 4.834)
    assert bench._profile_value(str(p), "psn::p3p_conv<512, 1,", "total_GB") == pytest.approx(4.834)
    assert bench._profile_value(str(p), "psn::p3p_conv<512, 1,", "read_GB") == pytest.approx(2.687)
    assert bench._profile_value(str(p), "psn::p4p_inv<512, 1,", "write_GB") == pytest.approx(1.074)


def test_profile_value_ignores_summaries_of_other_sources(tmp_path):
    p = tmp_path / "s.txt"
    _summary(p, "0000000000000000", 4.834)
    assert bench._profile_value(str(p), "psn::p3p_conv<512, 1,", "total_GB") is None
    assert bench._profile_value(str(tmp_path / "missing.txt"), "psn::p3p_conv<512, 1,", "total_GB") is None


def test_valu_roof_is_the_issue_rate():
    # 256 CUs, one wave64 VALU instruction per CU and cycle, 2.4 GHz
    assert bench.VALU_PEAK == pytest.approx(256 * 2.4e9)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr

"""Host logic of bench.py (CPU): the kernel-source digest that decides whether the committed
counter summaries still describe the kernel, and the readers of those summaries."""
import os
import shutil

import pytest

import bench


def test_region_takes_the_braced_block_or_the_statement():
    text = "int a;\nvoid f(int x) {\n  if (x) { g(); }\n}\nconstexpr int kB = 4;\nint z;\n"
    assert bench._region(text, "void f(") == "void f(int x) {\n  if (x) { g(); }\n}"
    assert bench._region(text, "constexpr int kB") == "constexpr int kB = 4;"
    with pytest.raises(ValueError):
        bench._region(text, "not in the text")


def _copy_sources(tmp_path, monkeypatch):
    for f, _ in [x for v in bench.KERNEL_SOURCES.values() for x in v]:
        dst = tmp_path / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(bench.ROOT, f), dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))


def test_digest_follows_kernel_regions_only(tmp_path, monkeypatch):
    d0 = bench.kernel_sources_digest()
    _copy_sources(tmp_path, monkeypatch)
    assert bench.kernel_sources_digest() == d0
    hip = tmp_path / "paper_2408_06765_amd/csrc/rsi_pairsum.hip"
    # host code outside the anchored regions leaves the digest alone
    hip.write_text(hip.read_text() + "\n// trailing note\n")
    assert bench.kernel_sources_digest() == d0
    # a change inside the kernel's definition changes it
    text = hip.read_text()
    i = text.index("pairsum_f32_kernel(")
    j = text.index("{", i) + 1
    hip.write_text(text[:j] + "\n    // edit\n" + text[j:])
    assert bench.kernel_sources_digest() != d0
    # the multi-frequency kernel's digest follows its own kernel only
    m0 = bench.kernel_sources_digest("multifreq")
    mf = tmp_path / "paper_2408_06765_amd/csrc/rsi_multifreq.hip"
    t2 = mf.read_text()
    k = t2.index("{", t2.index("multifreq_f32_kernel(")) + 1
    mf.write_text(t2[:k] + "\n    // edit\n" + t2[k:])
    assert bench.kernel_sources_digest("multifreq") != m0
    mf.write_text(t2)
    assert bench.kernel_sources_digest("multifreq") == m0
    # a moved anchor reads as stale counters, not as an error
    hip.write_text(text.replace("pairsum_f32_kernel(", "pairsum_f32_kernel_renamed("))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic() is None


def _summary(path, digest):
    path.write_text("# counters\n"
                    "traffic_bytes_per_launch: 123456\n"
                    "dipole_executed_fp32_tflops: 54.5\n"
                    "dipole_executed_fp32_frac: 0.35\n"
                    "dipole_valu_lane_util_pct: 100.0\n"
                    "dipole_cu_busy_pct: 99.0\n"
                    "dipole_issue_model_frac: 1.01\n"
                    f"kernel_sources_sha256: {digest}\n")


def test_summaries_are_read_only_while_the_digest_matches(tmp_path, monkeypatch):
    f = tmp_path / "summary.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    monkeypatch.setattr(bench, "VALU_FILE", str(f))
    _summary(f, bench.kernel_sources_digest())
    assert bench.measured_traffic() == 123456
    v = bench.measured_valu()
    assert v["executed_frac"] == 0.35 and v["issue_model_frac"] == 1.01
    _summary(f, "0" * 64)
    assert bench.measured_traffic() is None and bench.measured_valu() is None
    f.unlink()
    assert bench.measured_traffic() is None and bench.measured_valu() is None


def test_committed_summaries_parse():
    """The committed summaries carry the keys the readers use (whether or not they are
    current for the sources in this tree)."""
    for path, keys in ((bench.TRAFFIC_FILE, ["traffic_bytes_per_launch"]),
                       (bench.VALU_FILE, ["dipole_executed_fp32_frac", "dipole_cu_busy_pct"]),
                       (bench.MF_TRAFFIC_FILE, ["traffic_bytes_per_launch", "algorithmic_bytes_per_launch"]),
                       (bench.MF_VALU_FILE, ["dipole_executed_fp32_frac", "dipole_cu_busy_pct"])):
        text = open(path).read()
        assert "kernel_sources_sha256:" in text
        for k in keys:
            assert f"{k}:" in text


def test_flop_conventions():
    """The per-unit flop counts the roofline lines use: the ray pair through one plane (two
    Newton evaluations), one row of the surrogate network (128 frequencies, 5 x 256), and a
    multi-frequency dipole pair (33 for each block's first frequency, 21 per further one)."""
    assert bench.flops_ray_pair(2) == 104
    assert bench.flops_multifreq_pair(64) == 4 * 33 + 60 * 21
    assert bench.flops_multifreq_pair(20) == 2 * 33 + 18 * 21
    assert bench.flops_multifreq_pair(64, 32) == 2 * 33 + 62 * 21
    assert bench.flops_mlp_row(128, 256, 5) == 2 * (256 * 256 + 4 * 256 * 256 + 2 * 256)
    assert bench.FLOPS_DIPOLE == 33


def test_training_traffic_model():
    """The training step's HBM model: the library's split rule, and the bytes for the
    recipe's network (7 x 256 on 128 frequencies, 65536 rows) counted by hand: per row
    512 (features) + 2 (256 + 6 x 256) x 7 (forward) + 2560 (head and its gradient) +
    7 x 1536 + 6 x 2048 (backward); per step the split partials 2 x 4 x 128 x 458752 and
    the parameters 460290 x 24 plus 3 bf16 copies of the 458752 weights."""
    assert bench.dw_splits(65536) == 128
    assert bench.dw_splits(1000) == 4
    assert bench.dw_splits(64) == 1
    row = 512 + 7 * (2 * 256 + 6 * 256) + 2560 + 7 * 1536 + 6 * 2048
    weights = 7 * 256 * 256
    params = weights + 7 * 256 + 2 * 256 + 2
    step = 2 * 4 * 128 * weights + params * 24 + weights * 6
    assert bench.bytes_mlp_train_step(128, 256, 7, 65536, 128) == 65536 * row + step

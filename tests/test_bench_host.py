"""Host-side logic of the benchmark: the algorithmic byte counts of the two
passes and the kernel-source digest that decides whether committed counter
figures still describe the kernels."""
import os
import shutil

import pytest

import bench


def test_algorithmic_bytes_per_pixel():
    L = 4096
    row, col = bench.algorithmic_bytes(L, 4)
    spec = L * (L // 2 + 1) * 3 * 8            # half spectrum, 3 complex FP32 values per bin
    assert col == 2 * spec
    assert row == 2 * spec + 2 * 16 * L * L    # plus the stress state read and written
    assert row == 939720704
    # per pixel: 56 and 24 bytes (up to the extra Nyquist column)
    assert row / (L * L) == pytest.approx(56.0, rel=1e-3)
    assert col / (L * L) == pytest.approx(24.0, rel=1e-3)
    row64, col64 = bench.algorithmic_bytes(L, 8)
    assert row64 == 2 * row and col64 == 2 * col


def test_source_digest_ignores_comments_but_not_code(tmp_path, monkeypatch):
    src = os.path.join(bench.ROOT, "paper_0802_2488_amd", "csrc")
    dst = tmp_path / "paper_0802_2488_amd" / "csrc"
    dst.mkdir(parents=True)
    for name in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(src, name), dst / name)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    d0 = bench.kernel_sources_digest()
    k = dst / "pm_kernels.hpp"
    text = k.read_text()
    k.write_text("// a new line comment\n/* and a block\n comment */\n" + text.replace("\n", "\n\n", 3))
    assert bench.kernel_sources_digest() == d0
    k.write_text(text.replace("#define PM_ROW_PREFETCH 2", "#define PM_ROW_PREFETCH 3"))
    assert bench.kernel_sources_digest() != d0


def test_committed_counters_describe_the_current_kernels():
    """The counter summary under profiles/ was taken from the kernels as they
    are (its recorded source digest matches), and its HBM bytes per launch
    are within 20 % above the algorithmic bytes of each pass."""
    t = bench.measured_traffic()
    assert t is not None, "kernel sources changed since the counter summary was taken"
    row, col = bench.algorithmic_bytes(4096, 4)
    assert 1.0 <= t["k_row"] / row <= 1.2
    assert 1.0 <= t["k_column"] / col <= 1.2

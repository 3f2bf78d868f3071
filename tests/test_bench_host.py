"""Host helpers of the benchmark: the kernel code hash that ties the committed
counter profile to the kernel it was taken on."""
import bench


def test_code_text_ignores_comments_and_layout():
    a = "int f(int x) {\n  // one\n  return x + 1; /* two\n three */\n}\n"
    b = "int f(int x) { return x + 1; }"
    assert bench.code_text(a) == bench.code_text(b)
    assert bench.code_text(a) != bench.code_text("int f(int x) { return x + 2; }")


def test_kernel_source_hash_is_stable():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash()


def test_bench_refuses_more_than_one_gpu():
    """Several GPUs are refused with a message, before any GPU is touched."""
    import subprocess
    import sys
    res = subprocess.run([sys.executable, bench.__file__, "--gpus", "2"], capture_output=True, text=True,
                         timeout=300)
    assert res.returncode == 2
    assert "one GPU only" in res.stderr and res.stdout == ""


def test_bench_without_a_gpu_exits_with_a_message():
    """Without a visible GPU the benchmark stops with a message; it never falls
    back to another path."""
    import subprocess
    import sys

    import pytest
    from conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is visible")
    res = subprocess.run([sys.executable, bench.__file__, "--no-cpu"], capture_output=True, text=True, timeout=300)
    assert res.returncode == 2
    assert "needs an MI355X GPU" in res.stderr and res.stdout == ""

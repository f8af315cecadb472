"""The FLOP figure the benchmark reports equals the count taken from the
kernel's optimised device IR (compiled here, no GPU needed)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_flops_match_kernel_ir():
    sys.path.insert(0, ROOT)
    import bench
    from paper_2505_00097_amd import count_flops
    ir = count_flops.device_ir(os.path.join(ROOT, "paper_2505_00097_amd", "csrc", "rhs_fused.hip"))
    assert count_flops.count(ir) == bench.F_ALG
    assert count_flops.count(ir, dissipation=True, nghosts=5) == bench.F_ALG8_KO

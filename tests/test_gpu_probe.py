"""The FP64 FMA probe that bench.py uses to check the FP64 peak on the device."""
import pytest
import torch

import paper_2507_21686_amd as sb

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_fp64_fma_probe_counts_and_rate():
    sink = torch.zeros(1, dtype=torch.float64, device=DEV)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    f1 = sb.probe_fp64_fma(16, sink)
    assert f1 == 2 * 8 * 16 * n_cu * 8 * 256          # operations of the launch
    for _ in range(3):
        sb.probe_fp64_fma(4096, sink)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    flops = sum(sb.probe_fp64_fma(4096, sink) for _ in range(5))
    b.record()
    torch.cuda.synchronize()
    tflops = flops / (a.elapsed_time(b) * 1e-3) / 1e12
    print(f"FP64 FMA probe: {tflops:.1f} TFLOP/s on {n_cu} compute units", flush=True)
    assert 0.0 < tflops < 1.5 * 128 * n_cu * 2.4e9 / 1e12 * 1.2
    assert float(sink[0]) == 0.0                      # the guard store never happens
    with pytest.raises(sb.SphbiError, match="EINVAL"):
        sb.probe_fp64_fma(0, sink)

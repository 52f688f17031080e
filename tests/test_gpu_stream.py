"""The streaming driver on the device: an interrupted and resumed run reproduces the
accumulators of an uninterrupted one bit for bit, and equals one covariance call over
all images up to the FP32 partial-sum boundaries (norm-wise 1e-6)."""

import pytest
import torch

from paper_1412_0781_amd.stream import ChunkFailure, StreamConfig, run_on_device
from paper_1412_0781_amd.workload import synthetic_images

pytestmark = pytest.mark.gpu


def test_stream_resume_on_device(tmp_path):
    torch.cuda.set_device(0)
    cfg = StreamConfig(L=64, c=0.5, R=32.0, n=2500, chunk=1000, seed=2, snr=0.05, precision="bf16x3")
    print("[stream] uninterrupted", flush=True)
    plan, ref = run_on_device(cfg, checkpoint=str(tmp_path / "a.npz"))
    ck = str(tmp_path / "b.npz")
    print("[stream] interrupted at chunk 1", flush=True)
    with pytest.raises(ChunkFailure):
        run_on_device(cfg, checkpoint=ck, fail_at_chunk=1)
    print("[stream] resumed", flush=True)
    _, st = run_on_device(cfg, checkpoint=ck)
    assert st.count == ref.count == cfg.n
    assert torch.equal(st.G, ref.G) and torch.equal(st.S0, ref.S0)
    assert torch.equal(st.shift, ref.shift)
    x = synthetic_images(plan, 0, cfg.n, cfg.seed, cfg.snr)
    one = plan.new_covariance()
    one.shift.copy_(ref.shift)  # the shift the chunked run took from its first chunk
    one.shift_set = True
    plan.covariance(plan.expand(x, precision=cfg.precision), one, precision=cfg.precision)
    torch.cuda.synchronize()
    assert float((one.G - ref.G).norm() / one.G.norm()) <= 1e-6
    assert float((one.S0 - ref.S0).norm() / one.S0.norm()) <= 1e-6

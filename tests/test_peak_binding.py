"""The peak probes' Python binding refuses output buffers the kernels could
write past (host tensors, wrong dtype, fewer than n_blocks * 256 words) before
anything reaches the library (CPU only)."""
import pytest


def test_peak_binding_refuses_bad_buffers():
    import torch
    import paper_2309_03308_amd as pc
    with pytest.raises(ValueError):
        pc.corr_peak_mfma_f16(4, 1, torch.empty(4 * 256))  # a host tensor
    with pytest.raises(ValueError):
        pc.corr_peak_valu_f64(4, 1, torch.empty(4 * 256, dtype=torch.float32))  # wrong dtype
    with pytest.raises(ValueError):
        pc.corr_peak_hbm_read(torch.empty(64, dtype=torch.int32), 4, torch.empty(4 * 256, dtype=torch.int32))

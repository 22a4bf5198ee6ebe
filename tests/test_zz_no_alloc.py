"""The allocation-free learned-filter entry point (bf_lf_apply_noalloc) against bf_lf_apply,
through the C ABI: two calls in a row on the same device, the second on smaller images,
each bit-identical to bf_lf_apply on the same input (same kernels, same packed weights)."""
import numpy as np
import pytest

gpu = pytest.mark.gpu


@gpu
def test_lf_apply_noalloc_matches_apply_twice():
    import torch
    from paper_1009_2727_amd import LearnedFilter, bilinear_factor_params
    r = np.random.default_rng(31)
    params = (r.standard_normal(7200) * 0.05).astype(np.float32)
    params[:] += bilinear_factor_params(4, True)
    lf = LearnedFilter(params)
    for shape, per in (((3, 96, 130), (True, False)), ((2, 40, 52), (False, True))):
        x = torch.tensor(r.standard_normal(shape).astype(np.float32), device="cuda")
        ref = lf.apply(x, periodic=per)
        out = torch.full_like(x, float("nan"))
        lf.apply_noalloc(x, out, periodic=per)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(a).all()
        np.testing.assert_array_equal(a, b)

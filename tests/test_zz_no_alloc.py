"""The allocation-free inference entry point (srg_infer_noalloc) against the
context-based srg_infer, through the C ABI: bit-for-bit equal outputs on two
calls in a row, the second with a smaller batch and a shorter profile (the
static scratch keeps the first call's weights and is rewritten), with the
trained parameters and then with other parameters; sizes beyond its maximum and
bad arguments are refused before anything runs."""
import numpy as np
import pytest

from paper_1510_07328_amd import lbm
from paper_1510_07328_amd import surrogate as S

pytestmark = pytest.mark.gpu


def profiles(B, L, seed):
    rng = np.random.default_rng(seed)
    n = 1 + 0.1 * rng.standard_normal((B, L))
    u = 0.05 * rng.standard_normal((B, L))
    tau = rng.uniform(0.51, 1.0, B)
    return np.stack([n, u], axis=1).astype(np.float32), tau.astype(np.float32)


def test_noalloc_inference_equals_context_inference(gpu):
    import torch

    params, _ = S.load_weights()
    other = params + np.float32(0.01) * np.random.default_rng(7).standard_normal(params.shape).astype(np.float32)
    for p in (params, other):
        p_d = torch.from_numpy(np.ascontiguousarray(p, dtype=np.float32)).cuda()
        for B, L, seed in ((48, 1024, 1), (5, 256, 2)):  # second call smaller in batch and length
            prof, tau = profiles(B, L, seed)
            prof_d, tau_d = torch.from_numpy(prof).cuda(), torch.from_numpy(tau).cuda()
            sur = S.Surrogate(B, L, params=p)
            ref = sur.infer(prof_d, tau_d).clone()
            torch.cuda.synchronize()
            sur.free()
            out = torch.full_like(prof_d, float("nan"))
            S.srg_infer_noalloc(p_d, prof_d, tau_d, out)
            torch.cuda.synchronize()
            print(f"B={B} L={L}: max |noalloc - srg_infer| = {float((out - ref).abs().max()):.3e}", flush=True)
            assert torch.equal(out, ref)


def test_noalloc_inference_refuses_sizes_beyond_its_maximum(gpu):
    import torch

    params, _ = S.load_weights()
    p_d = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).cuda()
    for B, L in ((2, 4224), (2, 192), (2, 64)):
        prof_d = torch.ones((B, 2, L), dtype=torch.float32, device="cuda")
        tau_d = torch.full((B,), 0.7, dtype=torch.float32, device="cuda")
        out = torch.empty_like(prof_d)
        with pytest.raises(lbm.LbmError) as ei:
            S.srg_infer_noalloc(p_d, prof_d, tau_d, out)
        assert ei.value.status == -1
    prof_d = torch.ones((2, 2, 256), dtype=torch.float32, device="cuda")
    tau_d = torch.full((2,), 0.7, dtype=torch.float32, device="cuda")
    with pytest.raises(lbm.LbmError):  # output aliasing the input
        S.srg_infer_noalloc(p_d, prof_d, tau_d, prof_d)

"""The shell sums without allocation (ppmb_shell_profile_noalloc) against
the allocating entry point, through the C ABI: bitwise equal on two calls
in a row, the second on a smaller grid with fewer shells (the static
workspace keeps the first call's contents, which must not leak into the
second)."""
import numpy as np
import pytest

from paper_1810_13416_amd import problems as pr

pytestmark = pytest.mark.gpu


def _pair(S, nbins, dr):
    import torch
    want = S.shell_profile(nbins, dr)
    out = torch.full((nbins * 8,), float("nan"), dtype=torch.float64, device=S.buffers[0].device)
    S.shell_profile_noalloc(out, nbins, dr)
    S.synchronize()
    return want, out.cpu().numpy().reshape(nbins, 8)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_shell_sums_equal_allocating_ones(prec):
    from paper_1810_13416_amd import ppmb
    P = ppmb.FP64 if prec == "fp64" else ppmb.FP32
    big = pr.config3(n=48)
    A = ppmb.Sim(big.params, P)
    A.set_state(big.state)
    A.step_auto(big.cfl, 2)
    want, got = _pair(A, 24, 1.0 / 24)
    assert np.all(np.isfinite(got)) and np.array_equal(want, got)
    small = pr.config3(n=24)
    B = ppmb.Sim(small.params, P)
    B.set_state(small.state)
    B.step_auto(small.cfl, 1)
    want2, got2 = _pair(B, 10, 0.1)
    assert np.all(np.isfinite(got2)) and np.array_equal(want2, got2)


def test_noalloc_rejects_a_workspace_overflow():
    from paper_1810_13416_amd import ppmb
    import torch
    prob = pr.config3(n=128)          # 4096 blocks: 4161 * 8 doubles per shell
    S = ppmb.Sim(prob.params, ppmb.FP32)
    S.set_state(prob.state)
    out = torch.zeros(1024 * 8, dtype=torch.float64, device="cuda:0")
    with pytest.raises(ppmb.PPMBError, match="-1"):
        S.shell_profile_noalloc(out, 1024, 1.0 / 512)
    S.shell_profile_noalloc(out, 64, 1.0 / 64)     # within the limit
    S.synchronize()

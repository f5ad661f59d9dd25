"""pd_objective_grad_noalloc (the allocation-free variant of pd_objective_grad)
against pd_objective_grad on the same inputs: two calls in a row, the second on
a smaller input, in every precision; identical kernels and tiling, so the
results must agree bit for bit.  Also the host-side limits (map count, scratch
size), which are checked before any launch."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _case(pdl, rng, H, W, N, d, eps):
    import oracle
    lab = synth.random_labels(H, W, N, rng)
    th = synth.random_theta(N, d, rng, scale=0.4, multi_index=oracle.multi_index(d))
    p = pdl.Problem(torch.as_tensor(lab).cuda(), H, W, N, d, eps)
    return p, torch.as_tensor(th).cuda()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_noalloc_matches_objective_grad(pd, prec):
    pdl, ctx = pd
    rng = np.random.default_rng(7100)
    big = [_case(pdl, rng, 300, 421, 150, 4, 1e-2), _case(pdl, rng, 64, 200, 70, 3, 5e-2)]
    small = [_case(pdl, rng, 37, 70, 12, 2, 5e-2)]
    for batch in (big, small):
        probs = [b[0] for b in batch]
        ths = [b[1] for b in batch]
        print(f"noalloc {prec}: maps {[(p.H, p.W, p.N, p.d) for p in probs]}", flush=True)
        phi_ref, g_ref = ctx.objective_grad(probs, ths, prec)
        phi = torch.full((len(probs),), float("nan"), dtype=torch.float64, device="cuda")
        g = [torch.full_like(t, float("nan")) for t in ths]
        ctx.objective_grad_noalloc(probs, ths, phi, g, prec)
        torch.cuda.synchronize()
        assert torch.equal(phi, phi_ref), (phi, phi_ref)
        for a, b in zip(g, g_ref):
            assert torch.equal(a, b)
        # without the gradient
        phi2 = torch.zeros_like(phi)
        ctx.objective_grad_noalloc(probs, ths, phi2, None, prec)
        torch.cuda.synchronize()
        assert torch.equal(phi2, phi_ref)


def test_noalloc_limits(pd):
    pdl, ctx = pd
    rng = np.random.default_rng(7101)
    cases = [_case(pdl, rng, 16, 16, 3, 1, 0.1) for _ in range(pdl.NOALLOC_MAX_MAPS + 1)]
    probs = [c[0] for c in cases]
    ths = [c[1] for c in cases]
    phi = torch.zeros(len(probs), dtype=torch.float64, device="cuda")
    with pytest.raises(pdl.PdError) as e:
        ctx.objective_grad_noalloc(probs, ths, phi, None, "fp64")
    assert "at most" in str(e.value)
    # a map whose scratch does not fit: rejected before any launch
    lab = torch.zeros(2048 * 2048, dtype=torch.int32, device="cuda")
    p = pdl.Problem(lab, 2048, 2048, 4000, 6, 1e-3)
    th = torch.zeros((4000, 28), dtype=torch.float64, device="cuda")
    with pytest.raises(pdl.PdError) as e:
        ctx.objective_grad_noalloc([p], [th], phi[:1], None, "fp64")
    assert "scratch" in str(e.value)

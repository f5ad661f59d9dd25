"""pd_recover_params against the oracle's recovery (Section 5.6.3) on fitted
degree-1 and degree-2 coefficients, in the fit's gauge theta_N = 0."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


@pytest.mark.parametrize("kind", ["pd", "apd"])
def test_recover_matches_oracle_on_a_fit(pd, orc, kind):
    pdl, ctx = pd
    rng = np.random.default_rng(70)
    if kind == "pd":
        gm, d = synth.power_diagram(64, 64, 14, rng), 1
    else:
        gm, d = synth.anisotropic_power_diagram(64, 80, 16, rng), 2
    K = pdl.num_features(d)
    p = pdl.Problem(dev(gm.labels, torch.int32), gm.H, gm.W, gm.N, d, 1e-2)
    th = torch.zeros((gm.N, K), dtype=torch.float64, device="cuda")
    rep = ctx.fit([p], [th], "fp64", init="zero", max_iter=400, target_acc=0.99)[0]
    print(kind, rep["status"], rep["iters"], rep["acc"])
    x = th.cpu().numpy()
    assert np.all(x[-1] == 0.0)  # the fit's gauge: the last grain's anisotropy is 0
    out, lam = ctx.recover_params(th, d, margin=0.05)
    y, w, A, lam_ref = orc.recover_params(x, d, margin=0.05)
    o = out.cpu().numpy()
    if d == 2:
        assert lam_ref > 0.0
    assert abs(float(lam[0]) - lam_ref) <= 1e-12 * max(1.0, abs(lam_ref))
    scale = max(1.0, float(np.max(np.abs(y))))
    assert np.max(np.abs(o[:, 0:2] - y)) <= 1e-10 * scale
    assert np.max(np.abs(o[:, 2] - w)) <= 1e-10 * max(1.0, float(np.max(np.abs(w))))
    assert np.max(np.abs(o[:, 3] - A[:, 0, 0])) <= 1e-12 * max(1.0, float(np.max(np.abs(A))))
    assert np.max(np.abs(o[:, 4] - A[:, 0, 1])) <= 1e-12 * max(1.0, float(np.max(np.abs(A))))
    assert np.max(np.abs(o[:, 5] - A[:, 1, 1])) <= 1e-12 * max(1.0, float(np.max(np.abs(A))))
    if d == 2:
        Ad = np.empty((gm.N, 2, 2))
        Ad[:, 0, 0], Ad[:, 0, 1], Ad[:, 1, 0], Ad[:, 1, 1] = o[:, 3], o[:, 4], o[:, 4], o[:, 5]
        lmin = np.linalg.eigvalsh(Ad)[:, 0]
        assert np.all(lmin >= 0.05 - 1e-9)


def test_recover_errors(pd):
    pdl, ctx = pd
    th = torch.zeros((4, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(pdl.PdError):
        ctx.recover_params(th, 3)
    with pytest.raises(pdl.PdError):
        ctx.recover_params(torch.zeros((4, 6), dtype=torch.float64, device="cuda"), 2, margin=0.0)

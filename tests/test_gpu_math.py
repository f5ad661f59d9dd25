"""The evaluation kernels' elementary functions against the host's libm (numpy):
the FP64 2^x of the FP64 path (arguments <= 0, as the kernels form them) within
1 ulp, exact at integers, 0 below the subnormal range; the FP32 hardware 2^x and
log2 within their documented few ulps of FP32."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def ulps(got, ref):
    return np.abs(got - ref) / np.spacing(np.abs(ref))


def test_fp64_exp2_within_one_ulp(pd):
    pdl, ctx = pd
    rng = np.random.default_rng(0)
    x = np.concatenate([-rng.uniform(0, 1, 100000), -rng.uniform(0, 60, 100000),
                        -rng.uniform(0, 1000, 50000), -np.arange(0, 1023, dtype=np.float64),
                        [-0.5, -1.5, -2.5, -1e-300, -0.0, 0.0]])
    y = ctx.probe_math("exp2_f64", torch.as_tensor(x).cuda()).cpu().numpy()
    ref = np.exp2(x)
    u = ulps(y, ref)
    print(f"FP64 exp2: max {u.max():.3f} ulp, mean {u.mean():.3f}, exact {np.mean(y == ref):.3f}")
    assert u.max() <= 1.0
    ints = -np.arange(0, 1023, dtype=np.float64)
    yi = ctx.probe_math("exp2_f64", torch.as_tensor(ints).cuda()).cpu().numpy()
    assert np.array_equal(yi, np.exp2(ints))
    tiny = ctx.probe_math("exp2_f64", torch.as_tensor(np.array([-1080.0, -1100.0, -5000.0])).cuda()).cpu().numpy()
    assert np.all(tiny == 0.0)
    nan = ctx.probe_math("exp2_f64", torch.as_tensor(np.array([np.nan])).cuda()).cpu().numpy()
    assert np.isnan(nan[0])


def test_fp32_exp2_and_logs(pd):
    pdl, ctx = pd
    rng = np.random.default_rng(1)
    x = -rng.uniform(0, 100, 100000)
    y = ctx.probe_math("exp2_f32", torch.as_tensor(x).cuda()).cpu().numpy()
    ref = np.exp2(x.astype(np.float32)).astype(np.float64)
    ok = ref > np.finfo(np.float32).tiny
    uf = np.abs(y - ref)[ok] / np.spacing(ref[ok].astype(np.float32)).astype(np.float64)
    print(f"FP32 exp2: max {uf.max():.2f} ulp (normal range)")
    assert uf.max() <= 2.0
    z = rng.uniform(1e-3, 1e4, 100000)
    l64 = ctx.probe_math("log2_f64", torch.as_tensor(z).cuda()).cpu().numpy()
    assert np.max(ulps(l64, np.log2(z))[np.abs(np.log2(z)) > 1e-3]) <= 1.0
    l32 = ctx.probe_math("log2_f32", torch.as_tensor(z).cuda()).cpu().numpy()
    r32 = np.log2(z.astype(np.float32)).astype(np.float64)
    big = np.abs(r32) > 0.5
    u32 = np.abs(l32 - r32)[big] / np.spacing(r32[big].astype(np.float32)).astype(np.float64)
    print(f"FP32 log2: max {u32.max():.2f} ulp (|log2| > 0.5)")
    assert u32.max() <= 2.0

"""The C oracle under the host AddressSanitizer and UndefinedBehaviorSanitizer.

tests/sanitize/oracle_driver.c calls every exported oracle function on small
problems (among them a 1 x 1 map with two grains, the largest grid degree, a
NaN score); built with -fsanitize=address,undefined (any report aborts the run,
leaks included) it must exit cleanly and return, bit for bit, what the ordinary
build of the oracle returns for the same inputs.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DRIVER = os.path.join(HERE, "sanitize", "oracle_driver.c")
SRC = os.path.join(ROOT, "oracle", "pd_oracle.c")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_driver")
    cmd = ["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           DRIVER, SRC, "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("no sanitizer runtime: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr
    return exe


CASES = [  # H, W, N, d, D, points, theta scale, NaN entry
    (13, 17, 7, 3, 3, 200, 0.5, False),
    (5, 9, 3, 8, 2, 31, 0.2, False),
    (1, 1, 2, 1, 2, 1, 1.0, False),
    (6, 4, 5, 2, 3, 40, 0.5, True),
]


@pytest.mark.parametrize("case", CASES)
def test_sanitized_oracle_matches_ordinary_build(driver, tmp_path, case):
    H, W, N, d, D, npts, sc, with_nan = case
    rng = np.random.default_rng(H * 1000 + N)
    L = oracle._load()
    K = L.orc_num_features(d)
    Kp = L.orc_points_num_features(D, d)
    n = H * W
    eps = 0.05
    theta = rng.normal(scale=sc, size=(N, K))
    if with_nan:
        theta[1, 0] = np.nan
    labels = rng.integers(0, N, size=n).astype(np.int32)
    X = rng.uniform(-1.0, 1.0, size=(npts, D))
    theta_p = rng.normal(scale=sc, size=(N, Kp))
    labels_p = rng.integers(0, N, size=npts).astype(np.int32)
    inp, outp = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(inp, "wb") as f:
        f.write(np.array([H, W, N, d, D, npts], np.int32).tobytes())
        f.write(np.array([eps], np.float64).tobytes())
        for a in (theta, labels, X, theta_p, labels_p):
            f.write(np.ascontiguousarray(a).tobytes())
    supp = tmp_path / "lsan.supp"
    supp.write_text("leak:libgomp\n")
    # the same thread count as this process's oracle: the row-band sums are
    # combined per thread
    env = dict(os.environ, OMP_NUM_THREADS=str(L.orc_num_threads()),
               ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               LSAN_OPTIONS=f"suppressions={supp}",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([driver, str(inp), str(outp)], capture_output=True, text=True, env=env,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    buf = outp.read_bytes()
    pos = 0

    def read(dtype, count):
        nonlocal pos
        a = np.frombuffer(buf, dtype=dtype, count=count, offset=pos)
        pos += a.nbytes
        return a

    # the ordinary build, same calls
    A = np.zeros(64, np.int32)
    B = np.zeros(64, np.int32)
    L.orc_multi_index(d, A, B)
    assert np.array_equal(read(np.int32, K), A[:K]) and np.array_equal(read(np.int32, K), B[:K])
    assert read(np.float64, 1)[0] == L.orc_coord(3, W)
    P = np.zeros(d + 1)
    L.orc_legendre(-0.3, d, P)
    assert np.array_equal(read(np.float64, d + 1), P)
    feat = np.zeros(K * n)
    L.orc_features(H, W, d, feat)
    assert np.array_equal(read(np.float64, K * n), feat)
    g = np.zeros(N * K)
    phi = L.orc_objective_grad(H, W, N, d, eps, theta.ravel(), labels, g.ctypes.data)
    assert np.array_equal(read(np.float64, 1), [phi], equal_nan=True)
    assert np.array_equal(read(np.float64, N * K), g, equal_nan=True)
    b0, b1, a0 = (1, H - 1, 2) if H > 2 else (0, H, 0)
    v = L.orc_objective_grad_rows(H, W, N, d, eps, theta.ravel(), labels, b0, b1, g.ctypes.data)
    assert np.array_equal(read(np.float64, 1), [v], equal_nan=True)
    assert np.array_equal(read(np.float64, N * K), g, equal_nan=True)
    F = np.zeros(n, np.int32)
    nc = ctypes.c_int64(0)
    nn = L.orc_assign(H, W, N, d, theta.ravel(), labels.ctypes.data, F, ctypes.byref(nc))
    assert np.array_equal(read(np.int32, n), F)
    assert read(np.int64, 1)[0] == nc.value and read(np.int64, 1)[0] == nn
    assert (nn > 0) == with_nan
    rows = H - a0
    L.orc_assign_rows(H, W, N, d, theta.ravel(), labels.ctypes.data, a0, H, F, ctypes.byref(nc))
    assert np.array_equal(read(np.int32, rows * W), F[:rows * W])
    assert read(np.int64, 1)[0] == nc.value
    fp = np.zeros(Kp * npts)
    L.orc_points_features(npts, D, d, np.ascontiguousarray(X), fp)
    assert np.array_equal(read(np.float64, Kp * npts), fp)
    Fp = np.zeros(npts, np.int32)
    L.orc_points_assign(npts, D, N, d, theta_p.ravel(), np.ascontiguousarray(X),
                        labels_p.ctypes.data, Fp, ctypes.byref(nc))
    assert np.array_equal(read(np.int32, npts), Fp)
    assert read(np.int64, 1)[0] == nc.value
    assert pos == len(buf)

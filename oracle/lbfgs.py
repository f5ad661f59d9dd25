"""Oracle fit: limited-memory BFGS on -Phi with a strong-Wolfe line search, and a
dense damped Newton solve for tiny non-separable problems.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 5.2 fixes the protocol: start from theta = 0 (the fully ambiguous
diagram), maximise Phi with L-BFGS [Liu and Nocedal 1989], gauge fixed by
theta_N = 0 (Remark 4.3), a fixed iteration budget.  The paper names no memory
size, line search or tolerance; this oracle takes memory m = 10, initial inverse
Hessian gamma*I with gamma = s.y / y.y, a first trial step 1/||g||_2 when the
memory is empty and 1 otherwise, and the strong-Wolfe bracketing/zoom line search
of Nocedal and Wright (Algorithms 3.5 and 3.6) with c1 = 1e-4, c2 = 0.9, cubic
interpolation, doubling extrapolation and at most 20 evaluations per search.
A pair (s, y) is stored only when s.y > 1e-10 ||s|| ||y||.  A failed search
clears the memory and retries once from steepest descent.  The fit stops at the
first accepted iterate whose hard-assignment accuracy reaches the target, at the
iteration budget, or when ||g||_inf <= gtol.
"""
from __future__ import annotations

import math

import numpy as np

C1 = 1e-4
C2 = 0.9
MAX_LS_EVALS = 20
CURV_EPS = 1e-10


def _cubic_min(a, fa, da, b, fb, db):
    """Minimiser of the cubic interpolating (a, fa, da), (b, fb, db)
    (Nocedal and Wright eq. 3.59), kept inside the middle 80% of [a, b];
    bisection when the cubic has no admissible minimiser."""
    lo, hi = min(a, b), max(a, b)
    width = hi - lo
    mid = 0.5 * (a + b)
    d1 = da + db - 3.0 * (fa - fb) / (a - b)
    disc = d1 * d1 - da * db
    if not (disc >= 0.0):
        return mid
    d2 = math.copysign(math.sqrt(disc), b - a)
    den = db - da + 2.0 * d2
    if den == 0.0:
        return mid
    t = b - (b - a) * ((db + d2 - d1) / den)
    if not (lo + 0.1 * width <= t <= hi - 0.1 * width):
        return mid
    return t


def _line_search(evalf, x, f0, g0, d, t1):
    """Strong-Wolfe search along d from x.  evalf(x) -> (f, g).  Returns
    (ok, t, x_t, f_t, g_t, n_evals)."""
    dphi0 = float(g0.ravel() @ d.ravel())
    evals = 0
    best = None  # (t, x, f, g, dphi) with sufficient decrease, lowest f

    def trial(t):
        xt = x + t * d
        ft, gt = evalf(xt)
        return xt, ft, gt, float(gt.ravel() @ d.ravel())

    def zoom(lo, hi):
        nonlocal evals
        while evals < MAX_LS_EVALS:
            t = _cubic_min(lo[0], lo[2], lo[4], hi[0], hi[2], hi[4])
            xt, ft, gt, dt = trial(t)
            evals += 1
            if ft > f0 + C1 * t * dphi0 or ft >= lo[2]:
                hi = (t, xt, ft, gt, dt)
            else:
                if abs(dt) <= -C2 * dphi0:
                    return True, (t, xt, ft, gt, dt)
                if dt * (hi[0] - lo[0]) >= 0.0:
                    hi = lo
                lo = (t, xt, ft, gt, dt)
        return False, lo

    prev = (0.0, x, f0, g0, dphi0)
    t = t1
    while evals < MAX_LS_EVALS:
        xt, ft, gt, dt = trial(t)
        evals += 1
        cur = (t, xt, ft, gt, dt)
        if ft > f0 + C1 * t * dphi0 or (evals > 1 and ft >= prev[2]):
            ok, res = zoom(prev, cur)
            break
        if abs(dt) <= -C2 * dphi0:
            ok, res = True, cur
            break
        if dt >= 0.0:
            ok, res = zoom(cur, prev)
            break
        prev = cur
        t = 2.0 * t
    else:
        ok, res = False, prev
    if not ok:
        # fall back to the lowest point that still has sufficient decrease
        if res[0] > 0.0:
            ok = True
        best = res
    else:
        best = res
    t, xt, ft, gt, _ = best
    return ok, t, xt, ft, gt, evals


def lbfgs_fit(objective, theta0, *, accuracy=None, target_acc=0.99, max_iter=2000,
              history=10, gauge="last", gtol=0.0, callback=None, precondition=None,
              diag_every=10, diag_floor=1e-6):
    """Maximise Phi (minimise f = -Phi) from theta0.

    objective(theta) -> (Phi, grad Phi);  accuracy(theta) -> Acc in [0, 1] or None.
    precondition(theta) -> the diagonal of the Hessian of -Phi (N x K, eq. hess):
    if given, the initial inverse Hessian of the two-loop recursion is
    gamma * diag(1 / (D + diag_floor * max D)) instead of gamma * I, with D taken at
    the start and at every diag_every-th accepted iterate, gamma = s.y / y.D^-1 y
    of the newest pair (1 with an empty memory), and every search starts at t = 1
    (the last grain's row stays 0: gauge "last" only).
    Returns a dict with theta, phi, acc, iters, evals, status and per-iteration
    records (phi, acc, evals, t) for trajectory comparisons.
    """
    from . import gauge_project

    x = gauge_project(theta0, gauge) if gauge == "centered" else np.array(theta0, np.float64)
    if gauge == "last":
        # the common shift -theta_{N-1} puts the start in the gauge theta_{N-1} = 0
        # without changing Phi or the diagram (Lemma 4.2)
        x = x - x[-1]

    n_evals = 0

    def evalf(xx):
        nonlocal n_evals
        n_evals += 1
        phi, g = objective(xx)
        return -phi, gauge_project(-g, gauge)

    if precondition is not None and gauge != "last":
        raise ValueError("the diagonal preconditioner keeps gauge 'last'")
    Dinv = None

    def refresh(xx):
        D = np.asarray(precondition(xx), np.float64)
        Di = 1.0 / (D + diag_floor * float(np.max(D)))
        Di[-1, :] = 0.0
        return Di

    f, g = evalf(x)
    if precondition is not None:
        Dinv = refresh(x)
    S, Y, R = [], [], []
    gamma = 1.0
    it = 0
    records = []
    acc = accuracy(x) if accuracy is not None else None
    status = "budget"
    if acc is not None and acc >= target_acc:
        status = "target"
        return dict(theta=x, phi=-f, acc=acc, iters=0, evals=n_evals, status=status,
                    records=records)
    steep = (lambda gg: -gg) if Dinv is None else (lambda gg: -Dinv * gg)
    d = steep(g)
    reset_tried = False
    while it < max_iter:
        gnorm = float(np.sqrt(np.sum(g * g)))
        if gnorm == 0.0 or float(np.max(np.abs(g))) <= gtol:
            status = "gtol"
            break
        t1 = 1.0 / gnorm if (not S and Dinv is None) else 1.0
        dphi0 = float(g.ravel() @ d.ravel())
        if not (dphi0 < 0.0):
            S, Y, R = [], [], []
            d = steep(g)
            t1 = 1.0 / gnorm if Dinv is None else 1.0
        ok, t, xt, ft, gt, ev = _line_search(evalf, x, f, g, d, t1)
        if not ok:
            if S and not reset_tried:
                S, Y, R = [], [], []
                d = steep(g)
                reset_tried = True
                continue
            status = "linesearch"
            break
        reset_tried = False
        s = t * d
        y = gt - g
        sy = float(s.ravel() @ y.ravel())
        stored = sy > CURV_EPS * math.sqrt(float(s.ravel() @ s.ravel())) * math.sqrt(float(y.ravel() @ y.ravel()))
        if stored:
            if len(S) == history:
                S.pop(0), Y.pop(0), R.pop(0)
            S.append(s)
            Y.append(y)
            R.append(1.0 / sy)
        x, f, g = xt, ft, gt
        it += 1
        if Dinv is not None and it % diag_every == 0:
            Dinv = refresh(x)
        if stored:
            yDy = float(y.ravel() @ y.ravel()) if Dinv is None else float(np.sum(y * Dinv * y))
            gamma = sy / yDy
        acc = accuracy(x) if accuracy is not None else None
        records.append(dict(phi=-f, acc=acc, evals=ev, t=t))
        if callback is not None:
            callback(it, x, -f, acc)
        if acc is not None and acc >= target_acc:
            status = "target"
            break
        # two-loop recursion: d = -H g
        q = g.copy()
        alphas = []
        for sj, yj, rj in zip(reversed(S), reversed(Y), reversed(R)):
            a = rj * float(sj.ravel() @ q.ravel())
            alphas.append(a)
            q = q - a * yj
        r = (gamma if S else 1.0) * (q if Dinv is None else Dinv * q)
        for (sj, yj, rj), a in zip(zip(S, Y, R), reversed(alphas)):
            b = rj * float(yj.ravel() @ r.ravel())
            r = r + (a - b) * sj
        d = -r
    return dict(theta=x, phi=-f, acc=acc, iters=it, evals=n_evals, status=status,
                records=records)


def newton_fit(theta0, objective, hessian, *, gauge_last=True, tol=1e-12, max_iter=100):
    """Damped Newton ascent of Phi on the gauge-fixed subspace theta_N = 0
    (Proposition 4.11 gives a unique maximiser there when no exact reconstruction
    exists).  objective(theta) -> (Phi, grad); hessian(theta) -> (NK x NK)."""
    x = np.array(theta0, np.float64)
    N, K = x.shape
    if gauge_last:
        x[-1, :] = 0.0
    free = np.arange((N - 1) * K) if gauge_last else np.arange(N * K)
    for _ in range(max_iter):
        phi, g = objective(x)
        gv = g.reshape(-1)[free]
        if np.max(np.abs(gv)) <= tol:
            break
        Hm = hessian(x)[np.ix_(free, free)]
        step = np.linalg.solve(Hm, -gv)  # ascent direction for concave Phi
        t = 1.0
        while t > 1e-12:
            xn = x.copy()
            xn.reshape(-1)[free] += t * step
            if objective(xn)[0] >= phi + 1e-4 * t * float(gv @ step):
                break
            t *= 0.5
        x = xn
    return x


def annealed_fit(objective_eps, theta0, eps, *, stages, factor, stage_iters, accuracy=None,
                 target_acc=0.99, max_iter=2000, **fit_kw):
    """The fit with a decreasing schedule of the regularisation parameter, the
    annealing that Section 5.2 and the end of Section 5.6.4 leave to future work:
    eps_k = eps * factor**(stages - k), k = 0 .. stages, each level maximising
    Phi_{eps_k} with lbfgs_fit from the previous level's final theta (a new
    L-BFGS memory per level, since the curvature of Phi_eps scales with 1/eps^2).
    Levels k < stages run at most stage_iters iterations; the last one runs the
    rest of the max_iter budget.  Stopping is aligned with Err: the hard assignment
    F_theta does not depend on eps (Lemma 4.1 and the end of Section 5.6.4), so the
    first accepted iterate of any level with Acc >= target_acc ends the whole fit.

    objective_eps(theta, e) -> (Phi_e(theta), grad).  Returns lbfgs_fit's dict for
    the whole run (iters and evals summed over the levels; status of the last
    level; phi = Phi_eps at the final theta, at the target eps whichever level
    stopped) plus "levels": per level (eps_k, iters, evals, status, acc)."""
    if stages < 0 or not (factor > 1.0) or stage_iters < 0:
        raise ValueError("stages >= 0, factor > 1, stage_iters >= 0")
    x = np.array(theta0, np.float64)
    levels, records = [], []
    iters = evals = 0
    res = None
    for k in range(stages + 1):
        e_k = eps * factor ** (stages - k)
        budget = max_iter - iters if k == stages else min(stage_iters, max_iter - iters)
        res = lbfgs_fit(lambda th, e=e_k: objective_eps(th, e), x, accuracy=accuracy,
                        target_acc=target_acc, max_iter=budget, **fit_kw)
        x = res["theta"]
        iters += res["iters"]
        evals += res["evals"]
        records.extend(res["records"])
        levels.append(dict(eps=e_k, iters=res["iters"], evals=res["evals"],
                           status=res["status"], acc=res["acc"]))
        if res["status"] in ("target", "nonfinite") or iters >= max_iter and k < stages:
            if res["status"] != "target" and k < stages:
                res = dict(res, status="budget")
            break
    phi = res["phi"] if levels[-1]["eps"] == eps else float(objective_eps(x, eps)[0])
    return dict(theta=x, phi=phi, acc=res["acc"], iters=iters, evals=evals,
                status=res["status"], records=records, levels=levels)


def newton_cg_fit(objective, hvp, theta0, *, accuracy=None, target_acc=0.99, max_iter=100,
                  cg_max=20, gtol=0.0, c1=1e-4, max_halvings=30):
    """Inexact Newton ascent of Phi with Hessian-vector products (eq. hess of
    Proposition 4.4), in the gauge theta_N = 0 (on that subspace the Hessian of
    -Phi is positive definite, Proposition 4.11).  Per iteration: g = grad(-Phi)
    with its last row zeroed; conjugate gradients on H d = -g from d = 0, H the
    Hessian of -Phi (hvp(theta, v) -> H v, last row zeroed), stopped after cg_max
    steps, when ||r|| <= eta ||g|| with eta = min(0.5, sqrt(||g||)) (the forcing
    term of Eisenstat and Walker), or at non-positive curvature (d = -g if that
    happens at the first step); then step halving from t = 1 until
    -Phi(x + t d) <= -Phi(x) + c1 t g.d.  Stops at the first iterate (the start
    included) whose accuracy reaches target_acc, at max_iter iterations, when
    ||g||_inf <= gtol, or when the halving fails.
    Returns dict(theta, phi, acc, iters, evals, hvps, status, records)."""
    x = np.array(theta0, np.float64)
    x = x - x[-1]
    evals = hvps = 0
    records = []

    def f_g(xx):
        nonlocal evals
        evals += 1
        phi, g = objective(xx)
        g = -np.asarray(g, np.float64).copy()
        g[-1] = 0.0
        return -phi, g

    def H(v):
        nonlocal hvps
        hvps += 1
        w = np.asarray(hvp(x, v), np.float64).copy()
        w[-1] = 0.0
        return w

    f, g = f_g(x)
    acc = accuracy(x) if accuracy is not None else None
    status = "budget"
    it = 0
    while True:
        if acc is not None and acc >= target_acc:
            status = "target"
            break
        gn = math.sqrt(float(np.sum(g * g)))
        if gn == 0.0 or float(np.max(np.abs(g))) <= gtol:
            status = "gtol"
            break
        if it >= max_iter:
            break
        eta = min(0.5, math.sqrt(gn))
        d = np.zeros_like(g)
        r = -g
        p = r.copy()
        rr = float(np.sum(r * r))
        for k in range(cg_max):
            Hp = H(p)
            pHp = float(np.sum(p * Hp))
            if not (pHp > 0.0):
                if k == 0:
                    d = -g
                break
            alpha = rr / pHp
            d = d + alpha * p
            r = r - alpha * Hp
            rr_new = float(np.sum(r * r))
            if math.sqrt(rr_new) <= eta * gn:
                break
            p = r + (rr_new / rr) * p
            rr = rr_new
        gd = float(np.sum(g * d))
        t = 1.0
        for _ in range(max_halvings):
            fx, gx = f_g(x + t * d)
            if fx <= f + c1 * t * gd:
                break
            t *= 0.5
        else:
            status = "linesearch"
            break
        x = x + t * d
        f, g = fx, gx
        it += 1
        acc = accuracy(x) if accuracy is not None else None
        records.append(dict(phi=-f, acc=acc, t=t, cg=k + 1))
    return dict(theta=x, phi=-f, acc=acc, iters=it, evals=evals, hvps=hvps, status=status,
                records=records)

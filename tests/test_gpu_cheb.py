"""GPU parity of the Chebyshev smoother (the Chebyshev iteration for S A on
[cheb_lo, cheb_hi] * lambda, lambda by power iteration; a stronger smoother of the
fixed-matrix family, Sec. 6) against the oracle, through the C ABI.

Tolerances as for the damped (block-)Jacobi path: the eigenvalue estimate (FP64, norms
summed in another order) to 1e-12 relative; one smoothing phase to 1e-12 of the scale
|A||x| + |b| + |x| of its inputs (a few FP64 sweeps whose coefficients agree to
~1e-15); V-cycles to 1e-12 relative; converged solutions to 1e-10 relative with equal
cycle counts."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import hierarchy as Hh, multigrid as MG

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _log(*a):
    print("[gpu-cheb]", *a, flush=True)
    sys.stdout.flush()


def _cheb(wl, **kw):
    return wl.with_(smoother=W.SMOOTH_CHEBYSHEV, **kw)


CASES = {
    "poisson33": _cheb(W.c1_poisson(4)),
    "td_band": _cheb(W.c2_td(band_rounds=3, uniform_rounds=1), cheb_lo=0.3, cheb_hi=1.2),
    "elast17": _cheb(W.c3_elasticity(3)),
    "edge4": _cheb(W.c3_adaptive("edge", 4)),
    "elast17_23": _cheb(W.c3_elasticity(3), nu1=2, nu2=3),
}

_cache = {}


def _pair(name, precision="fp64"):
    key = (name, precision)
    if key not in _cache:
        from paper_2405_05047_amd import gen, mg
        wl = CASES[name]
        if name not in _cache:
            _log("building", name)
            o = Hh.build(wl)
            _cache[name] = (o, MG.Multigrid(o), gen.build(wl))
        o, mgo, p = _cache[name]
        h = mg.Hierarchy(p.levels, mg.config_from(wl, precision=precision))
        _cache[key] = (wl, o, mgo, p, h)
    return _cache[key]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_eigen_estimates_match(name):
    wl, o, mgo, p, h = _pair(name)
    for l in range(1, h.n_levels):
        lam = h.eigen_estimate(l)
        assert abs(lam - mgo.lam[l]) <= 1e-12 * mgo.lam[l], (l, lam, mgo.lam[l])


@pytest.mark.parametrize("name", list(CASES))
def test_smoothing_phase_parity(name):
    """nu steps from a seeded x and from 0 on every level >= 1."""
    wl, o, mgo, p, h = _pair(name)
    for l in range(1, len(o.levels)):
        lv = o.levels[l]
        A = lv.A
        x = W.rand_vec(300 + l, lv.ndof)
        b = W.rand_vec(400 + l, lv.ndof)
        scale = (abs(A) @ np.abs(x) + np.abs(b) + np.abs(x)).max()
        for k in sorted({1, wl.nu1, wl.nu2}):
            out = torch.empty(lv.ndof, dtype=torch.float64, device="cuda")
            h.smooth(l, dev(b), dev(x), out, sweeps=k)
            ref = mgo.chebyshev(l, x, b, k)
            assert np.abs(host(out) - ref).max() <= 1e-12 * scale, (l, k)
            h.smooth(l, dev(b), None, out, sweeps=k)
            ref = mgo.chebyshev(l, np.zeros_like(b), b, k)
            assert np.abs(host(out) - ref).max() <= 1e-12 * scale, (l, k, "from 0")


@pytest.mark.parametrize("name", list(CASES))
def test_vcycle_parity(name):
    wl, o, mgo, p, h = _pair(name)
    b = o.b
    x = torch.zeros(len(b), dtype=torch.float64, device="cuda")
    h.vcycle(dev(b), x)
    ref = mgo.vcycle(b)
    assert np.linalg.norm(host(x) - ref) <= 1e-12 * np.linalg.norm(ref)
    # GMG(L, x, b) from a nonzero iterate
    x0 = W.rand_vec(9, len(b))
    x = dev(x0)
    h.vcycle(dev(b), x, x_is_zero=False)
    ref = mgo.gmg(o.L, x0, b)
    assert np.linalg.norm(host(x) - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("name", list(CASES))
def test_solve_parity(name):
    wl, o, mgo, p, h = _pair(name)
    b = dev(o.b)
    x = torch.zeros_like(b)
    st = h.solve(b, x)
    xr, sr = mgo.solve(o.b)
    _log(name, "cycles", st["iters"], "oracle", sr.iters)
    assert st["converged"] == 1 and st["iters"] == sr.iters
    assert np.linalg.norm(host(x) - xr) <= 1e-10 * np.linalg.norm(xr)


@pytest.mark.parametrize("precision", ["fp32", "fp16"])
def test_mixed_precision_chebyshev_reaches_fp64_tolerance(precision):
    wl, o, mgo, p, h = _pair("elast17", precision)
    b = dev(o.b)
    x = torch.zeros_like(b)
    st = h.solve(b, x)
    xr, sr = mgo.solve(o.b)
    res = np.linalg.norm(o.b - o.finest.A @ host(x)) / np.linalg.norm(o.b)
    err = np.linalg.norm(host(x) - xr) / np.linalg.norm(xr)
    _log(precision, "cycles", st["iters"], "fp64 oracle", sr.iters, f"residual {res:.2e} error {err:.2e}")
    assert st["converged"] == 1 and res <= wl.rtol and err <= 1e-6


def test_batch_refuses_chebyshev():
    from paper_2405_05047_amd import mg
    wl, o, mgo, p, h = _pair("poisson33")
    with pytest.raises(mg.MGError):
        mg.Batch([p.levels], mg.config_from(wl.with_(outer=W.OUTER_FGMRES)), nrhs=1)

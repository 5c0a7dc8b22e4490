"""GPU parity of the reduced-precision form step by step (FP32 cycle; FP32, FP16 x 2^e
and BF16 x 2^e stored values), through the C ABI, against the oracle's FP32 emulation.

Each kernel step of the cycle is compared element by element with the exact value of
that step on the FP32 data the cycle holds (oracle.mixed: decoded stored values, the
FP64 block inverses rounded to FP32, omega rounded to FP32).  The tolerance per row is
the a-priori bound of evaluating the row's sums in FP32 (gamma_k sum |terms|,
u = 2^-24, k = terms in the row plus the roundings of the update), so a wrong code, a
wrong row exponent, a dropped term or a mis-scaled decode fails by far more than it.
The stored operator itself is compared bit for bit with the oracle codec.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import codec, hierarchy as Hh, mixed as MX, multigrid as MG

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FMTS = ["fp32", "fp16", "bf16"]
CASES = {
    "td_band": W.c2_td(band_rounds=3, uniform_rounds=1),
    "elast17": W.c3_elasticity(3),
    "oseen17": W.c4_oseen(3),
    "edge4": W.c3_adaptive("edge", 4),
}

_cache = {}


def _log(*a):
    print("[gpu-mixed]", *a, flush=True)
    sys.stdout.flush()


def _pair(name, fmt):
    from paper_2405_05047_amd import gen, mg
    key = (name, fmt)
    if key not in _cache:
        wl = CASES[name]
        if name not in _cache:
            _log("building", name)
            _cache[name] = (Hh.build(wl), gen.build(wl))
        o, p = _cache[name]
        _log("setup", name, fmt)
        h = mg.Hierarchy(p.levels, mg.config_from(wl, precision=fmt))
        _cache[key] = (wl, o, p, h)
    return _cache[key]


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def _rand32(seed, n):
    return MX.f32(W.rand_vec(seed, n))


def _terms(A):
    return np.diff(A.indptr)


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("name", list(CASES))
def test_stored_operator_bit_exact(name, fmt):
    """The library's stored values (FP32 roundings, or FP16 / BF16 codes and per-row
    exponents) equal the oracle codec bit for bit on every level, applied to the operator
    the library was given (the generator's assembly, which agrees with the oracle's only
    to FP64 rounding, so its FP32 / FP16 roundings may differ in a few entries)."""
    wl, o, p, h = _pair(name, fmt)
    for l, lv in enumerate(p.levels):
        vals, ex = h.export(l)
        A = MX.block_csr(lv)
        # the library exports in BSR order (block k, row c, column cc); the oracle's CSR
        # holds the same entries sorted by (scalar row, column)
        nb, b = lv.nnzb, wl.block
        rows = (np.repeat(np.arange(lv.n), np.diff(lv.rowptr))[:, None, None] * b
                + np.arange(b)[None, :, None] + 0 * np.arange(b)[None, None, :])
        cols = lv.col[:, None, None].astype(np.int64) * b + np.arange(b)[None, None, :] + 0 * rows
        order = np.lexsort((cols.ravel(), rows.ravel()))
        got = vals.reshape(nb * b * b)[order]
        if fmt == "fp32":
            assert np.array_equal(got.view(np.uint32), A.data.astype(np.float32).view(np.uint32)), (name, l)
        else:
            e_ref, q_ref = codec.encode(A, fmt)
            assert np.array_equal(ex.astype(np.int32), e_ref), (name, l, "exponents")
            assert np.array_equal(got, q_ref), (name, l, "codes")


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("name", list(CASES))
def test_spmv_defect_steps(name, fmt):
    wl, o, p, h = _pair(name, fmt)
    for l, lv in enumerate(o.levels):
        A32 = MX.stored_operator(lv, fmt)
        k = _terms(A32)
        x = _rand32(100 + l, lv.ndof)
        b = _rand32(200 + l, lv.ndof)
        ax = abs(A32) @ np.abs(x)
        y = torch.zeros(lv.ndof, dtype=torch.float32, device="cuda")
        h.spmv(l, dev32(x), y)
        ref = A32 @ x
        tol = MX.fp32_row_bound(k + 1, ax) + 1e-38
        assert np.all(np.abs(host(y) - ref) <= tol), (name, fmt, l, np.max(np.abs(host(y) - ref) / tol))
        r = torch.zeros_like(y)
        h.defect(l, dev32(b), dev32(x), r)
        ref = b - A32 @ x
        tol = MX.fp32_row_bound(k + 2, np.abs(b) + ax) + 1e-38
        assert np.all(np.abs(host(r) - ref) <= tol), (name, fmt, l, "defect")
        h.defect(l, dev32(b), dev32(x), r, masked=True)
        ref[lv.mask.ravel()] = 0.0
        got = host(r)
        assert np.all(got[lv.mask.ravel()] == 0.0)
        assert np.all(np.abs(got - ref) <= tol), (name, fmt, l, "masked defect")


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("name", list(CASES))
def test_sweep_steps(name, fmt):
    wl, o, p, h = _pair(name, fmt)
    for l, lv in enumerate(o.levels):
        A32 = MX.stored_operator(lv, fmt)
        S32 = MX.stored_smoother(lv)
        k = _terms(A32) + wl.block + 4
        x = _rand32(300 + l, lv.ndof)
        b = _rand32(400 + l, lv.ndof)
        om = MX.f32(wl.omega)
        mag = np.abs(x) + om * MX.apply_blocks(np.abs(S32), np.abs(b) + abs(A32) @ np.abs(x))
        xo = torch.zeros(lv.ndof, dtype=torch.float32, device="cuda")
        h.sweep(l, dev32(b), dev32(x), xo)
        ref = MX.sweep(A32, S32, wl.omega, x, b)
        tol = MX.fp32_row_bound(k, mag) + 1e-38
        assert np.all(np.abs(host(xo) - ref) <= tol), (name, fmt, l, np.max(np.abs(host(xo) - ref) / tol))
        h.sweep0(l, dev32(b), xo)
        ref0 = MX.sweep0(S32, wl.omega, b)
        tol0 = MX.fp32_row_bound(np.full(lv.ndof, wl.block + 2), om * MX.apply_blocks(np.abs(S32), np.abs(b))) + 1e-38
        assert np.all(np.abs(host(xo) - ref0) <= tol0), (name, fmt, l, "sweep0")


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("name", list(CASES))
def test_transfer_and_coarse_steps(name, fmt):
    wl, o, p, h = _pair(name, fmt)
    for l in range(1, len(o.levels)):
        f, c = o.levels[l], o.levels[l - 1]
        r = _rand32(500 + l, f.ndof)
        d = torch.zeros(c.ndof, dtype=torch.float32, device="cuda")
        h.restrict(l, dev32(r), d)
        ref = f.R @ r                                   # dyadic weights: exact in FP32
        tol = MX.fp32_row_bound(np.diff(f.R.indptr) + 1, abs(f.R) @ np.abs(r)) + 1e-38
        got = host(d)
        assert np.all(np.abs(got - ref) <= tol), (name, fmt, l, "restrict")
        assert np.all(got[c.mask.ravel()] == 0.0)
        y = _rand32(600 + l, c.ndof)
        x = _rand32(700 + l, f.ndof)
        xt = dev32(x)
        h.prolong(l, dev32(y), xt)
        ref = x + f.P @ y
        tol = MX.fp32_row_bound(np.diff(f.P.indptr) + 2, np.abs(x) + abs(f.P) @ np.abs(y)) + 1e-38
        assert np.all(np.abs(host(xt) - ref) <= tol), (name, fmt, l, "prolong")
    mgo = MG.Multigrid(o)
    b0 = _rand32(800, o.levels[0].ndof)
    b0[o.levels[0].mask.ravel()] = 0.0
    x0 = torch.zeros(len(b0), dtype=torch.float32, device="cuda")
    h.coarse_solve(dev32(b0), x0)
    ref = mgo.coarse_solve(b0)                          # FP64 inverse applied to the FP32 data
    tol = 2 * MX.U32 * np.abs(ref) + 1e-12 * np.abs(ref).max() * max(1.0, np.linalg.cond(mgo.A0) / 1e3)
    assert np.all(np.abs(host(x0) - ref) <= tol), (name, fmt, "coarse")


@pytest.mark.parametrize("fmt", FMTS)
@pytest.mark.parametrize("name", ["td_band", "elast17", "oseen17"])
def test_mixed_vcycle_close_to_fp64(name, fmt):
    """One whole V-cycle of the mixed form against the FP64 oracle V-cycle: the FP32 data
    perturb it by ~cond * u relative (FP16 / BF16 storage: by their unit roundoff)."""
    wl, o, p, h = _pair(name, fmt)
    ref = MG.Multigrid(o).vcycle(o.b)
    x = torch.zeros(len(o.b), dtype=torch.float64, device="cuda")
    h.vcycle(torch.from_numpy(o.b).cuda(), x)
    err = np.linalg.norm(host(x) - ref) / np.linalg.norm(ref)
    _log(name, fmt, "vcycle rel err vs fp64", err)
    assert err <= {"fp32": 1e-4, "fp16": 5e-2, "bf16": 2e-1}[fmt]
